// Host-only paths of the C ABI under AddressSanitizer and UndefinedBehavior-
// Sanitizer: parameter derivation and validation over seeded random, extreme
// and invalid parameter sets, buffer sizes, and the argument checks of every
// entry point that validates before it touches a GPU.  Prints "ok" and exits 0.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/rmrt.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void) {   // splitmix64
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static double uni(double lo, double hi) { return lo + (hi - lo) * (double)(next_u64() >> 11) / 9007199254740992.0; }
static int pick(int n) { return (int)(next_u64() % (uint64_t)n); }

static int failures = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                \
    }                                                            \
  } while (0)

static double odd_value(void) {
  const double v[] = {0.0, -1.0, 1e-300, 1e300, NAN, INFINITY, -INFINITY, 2.0, 0.5, 1e-12};
  return v[pick(10)];
}

int main(void) {
  const int lat[] = {RMRT_Q9, RMRT_Q19, RMRT_Q27, RMRT_Q5, RMRT_Q7};
  int ok_count = 0;
  for (int it = 0; it < 20000; ++it) {
    rmrt_params p;
    memset(&p, 0, sizeof(p));
    p.lattice = pick(7) == 0 ? pick(20) - 5 : lat[pick(5)];
    p.equation = pick(10) == 0 ? 7 : pick(2);
    p.storage = pick(10) == 0 ? -1 : pick(3);
    p.pattern = pick(10) == 0 ? 3 : pick(2);
    const int two_d = p.lattice == RMRT_Q9 || p.lattice == RMRT_Q5;
    for (int a = 0; a < 3; ++a) p.n[a] = pick(20) == 0 ? pick(3) - 1 : 1 + pick(300);
    if (two_d && pick(4)) p.n[2] = 1;
    if (pick(50) == 0) p.n[0] = p.n[1] = p.n[2] = 4096;   // beyond 32-bit indexing
    for (int a = 0; a < 3; ++a) {
      const double choices[] = {0.5, 1.0, 2.0};
      p.dx[a] = pick(20) == 0 ? odd_value() : choices[pick(3)];
    }
    p.dt = pick(10) == 0 ? odd_value() : 1.0;
    p.cs2 = pick(3) == 0 ? uni(0.01, 0.5) : (pick(10) == 0 ? odd_value() : -1.0);
    p.nu = pick(10) == 0 ? odd_value() : uni(1e-3, 0.3);
    p.nu_b = pick(3) == 0 ? -1.0 : (pick(10) == 0 ? odd_value() : uni(1e-3, 0.3));
    p.s_hi = pick(5) == 0 ? uni(0.1, 1.9) : (pick(10) == 0 ? odd_value() : -1.0);
    p.w_corner = pick(5) == 0 ? uni(0.0, 0.05) : -1.0;
    p.D0 = pick(10) == 0 ? odd_value() : uni(1e-3, 0.2);
    p.D2 = pick(10) == 0 ? odd_value() : uni(0.0, 2.0);
    for (int a = 0; a < 3; ++a) {
      p.adv[a] = uni(-0.1, 0.1);
      p.force[a] = uni(-1e-4, 1e-4);
    }
    p.source = pick(2) ? uni(-1e-3, 1e-3) : 0.0;
    p.rho0 = pick(10) == 0 ? odd_value() : 1.0;
    p.wall_faces = (unsigned)pick(64);
    p.check_every = pick(3);
    p.incompressible = pick(4) == 0;
    for (int k = 0; k < 6; ++k) p.nu_tensor[k] = pick(4) == 0 ? (pick(10) == 0 ? odd_value() : uni(1e-3, 0.2)) : -1.0;
    for (int k = 0; k < 3; ++k) p.nu_b_axis[k] = pick(4) == 0 ? uni(1e-3, 0.2) : -1.0;
    p.gamma0 = pick(4) == 0;
    p.diffusive = pick(6) == 0;
    p.c_zero = pick(4) == 0;
    p.central = pick(6) == 0;
    p.hermite = pick(6) == 0;
    p.bhll = pick(6) == 0;

    rmrt_derived d;
    const int rc = rmrt_derive(&p, &d);
    size_t bytes = 0;
    const int rb = rmrt_population_bytes(&p, &bytes);
    CHECK(rc == rb);
    CHECK(rc == RMRT_OK || rc == RMRT_EINVAL || rc == RMRT_EUNSUPPORTED);
    const char* msg = rmrt_last_error();
    CHECK(msg != NULL);
    if (rc == RMRT_OK) {
      ++ok_count;
      double wsum = 0.0;
      for (int j = 0; j < d.q; ++j) {
        CHECK(d.w[j] >= 0.0);
        wsum += d.w[j];
      }
      CHECK(fabs(wsum - 1.0) < 1e-12);
      CHECK(d.s_hi > 0.0 && d.s_hi < 2.0);
      CHECK(bytes >= (size_t)d.q * (size_t)p.n[0] * (size_t)p.n[1] * (size_t)p.n[2]);
    } else {
      CHECK(strlen(msg) > 0);
    }
  }
  CHECK(ok_count > 1000);

  // argument checks that return before any GPU work
  rmrt_params p;
  memset(&p, 0, sizeof(p));
  p.lattice = RMRT_Q9;
  p.n[0] = p.n[1] = 8;
  p.n[2] = 1;
  p.dx[0] = p.dx[1] = p.dx[2] = 1.0;
  p.nu = 0.1;
  p.nu_b = -1.0;
  p.w_corner = -1.0;
  p.rho0 = 1.0;
  CHECK(rmrt_derive(NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_derive(&p, NULL) == RMRT_EINVAL);
  CHECK(rmrt_population_bytes(&p, NULL) == RMRT_EINVAL);
  CHECK(rmrt_init(NULL, &p, NULL, NULL, NULL, NULL, NULL, 0, NULL) == RMRT_EINVAL);
  rmrt_ctx* ctx = NULL;
  CHECK(rmrt_init(&ctx, &p, NULL, NULL, NULL, NULL, NULL, 0, NULL) == RMRT_EINVAL);   // f0 NULL
  CHECK(ctx == NULL);
  CHECK(rmrt_step(NULL, 1, NULL) == RMRT_EINVAL);
  CHECK(rmrt_step_prepare(NULL, 1, NULL) == RMRT_EINVAL);
  CHECK(rmrt_set_fields(NULL, NULL, NULL, 0, NULL) == RMRT_EINVAL);
  CHECK(rmrt_set_source_fields(NULL, NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_moments(NULL, NULL, NULL, RMRT_OUT_F64, NULL) == RMRT_EINVAL);
  CHECK(rmrt_populations(NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_local_gradients(NULL, RMRT_GRAD_STRAIN, NULL, RMRT_OUT_F64, NULL) == RMRT_EINVAL);
  CHECK(rmrt_step_local(NULL, RMRT_GRAD_STRAIN, NULL, RMRT_OUT_F64, NULL) == RMRT_EINVAL);
  double out4[4];
  CHECK(rmrt_reduce(NULL, out4, NULL) == RMRT_EINVAL);
  CHECK(rmrt_reduce_noalloc(NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_residual(NULL, NULL, NULL) == RMRT_EINVAL);
  long long st;
  CHECK(rmrt_steps_taken(NULL, &st) == RMRT_EINVAL);
  size_t cb;
  CHECK(rmrt_checkpoint_bytes(NULL, &cb) == RMRT_EINVAL);
  CHECK(rmrt_checkpoint_save(NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_checkpoint_restore(NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_set_launch(NULL, 0, 0) == RMRT_EINVAL);
  CHECK(rmrt_get_launch(NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_tune(NULL, 1, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_free(NULL) == RMRT_OK);
  rmrt_batch* b = NULL;
  CHECK(rmrt_batch_create(NULL, 1, &p, NULL, NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_create(&b, 0, &p, NULL, NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_step(NULL, 1, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_step_prepare(NULL, 1, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_autotune(NULL, 1, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_set_config(NULL, 0) == RMRT_EINVAL);
  CHECK(rmrt_batch_set_group_bytes(NULL, 0) == RMRT_EINVAL);
  CHECK(rmrt_batch_get_group_bytes(NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_set_xcd_chunks(NULL, 1) == RMRT_EINVAL);
  CHECK(rmrt_batch_get_xcd_chunks(NULL, NULL, NULL) == RMRT_EINVAL);
  double growth = 0;
  CHECK(rmrt_preflight(NULL, NULL, 100, &growth, NULL) == RMRT_EINVAL);
  CHECK(rmrt_preflight(&p, NULL, 100, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_preflight(&p, NULL, 8, &growth, NULL) == RMRT_EINVAL);
  CHECK(rmrt_preflight(&p, NULL, 2000000, &growth, NULL) == RMRT_EINVAL);
  CHECK(rmrt_checked_build() == 0);
  unsigned oob = 0;
  CHECK(rmrt_checked_violations(NULL, &oob, NULL) == RMRT_EINVAL);
  CHECK(rmrt_checked_set_limit(NULL, 1, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_domain(NULL, 0, &ctx) == RMRT_EINVAL);
  CHECK(rmrt_batch_residual(NULL, NULL, NULL) == RMRT_EINVAL);
  CHECK(rmrt_batch_free(NULL) == RMRT_OK);
  const int nc = rmrt_batch_num_configs();
  CHECK(nc > 0);
  for (int c = -2; c < nc + 2; ++c) {
    int t, tn, bpc, per, npt;
    const int r = rmrt_batch_config_info(c, &t, &tn, &bpc, &per, &npt);
    CHECK((c >= 0 && c < nc) ? (r == RMRT_OK && t > 0 && t <= 256 && tn >= t) : r == RMRT_EINVAL);
  }
  CHECK(rmrt_version() != NULL && strlen(rmrt_version()) > 0);
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("ok %d valid parameter sets\n", ok_count);
  return 0;
}
