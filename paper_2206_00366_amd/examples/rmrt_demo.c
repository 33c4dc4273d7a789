/*
 * Plain-C use of the rmrt C ABI (no Python, no torch): a periodic rD3Q19
 * Taylor-Green vortex of small amplitude (U0 = 1e-3, the linear regime) on a
 * rectangular grid with dz = 2 dx, stepped in the AA pattern (eq. 2-2-3).  The
 * initial populations carry the non-equilibrium part of eq. fne, so the mode
 * decays at its viscous rate from the first step.  The program allocates the
 * populations and the initial fields with hipMalloc, initialises the context,
 * steps it, and prints, one "key value" line each:
 *   mass0 / mass1        FP64 sum of rho before and after the steps (eq. 4-18-1)
 *   mom1_x, mom1_y, mom1_z  FP64 momentum after the steps
 *   amp0 / amp1          projection of u on the initial mode
 *   nu_fit               -ln(amp1 / amp0) / (steps k^2): the decay rate of the
 *                        mode, which the method recovers as the viscosity nu
 *
 * Usage: rmrt_demo [steps (default 300)] [storage: 0 FP64, 1 FP32-dev, 2 FP16-dev]
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "rmrt.h"

#define HIP_OK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                      \
      return 1;                                                                    \
    }                                                                              \
  } while (0)
#define RMRT_OK_OR_EXIT(x)                                                         \
  do {                                                                             \
    int rc_ = (x);                                                                 \
    if (rc_ != RMRT_OK) {                                                          \
      fprintf(stderr, "%s: %d %s\n", #x, rc_, rmrt_last_error());                  \
      return 1;                                                                    \
    }                                                                              \
  } while (0)

static const double kPi = 3.14159265358979323846;

/* mode shape of the x velocity: sin(kx x) cos(ky y) cos(kz z) */
static double mode(const int n[3], const double dx[3], int i, int j, int k) {
  const double kx = 2 * kPi / (n[0] * dx[0]), ky = 2 * kPi / (n[1] * dx[1]), kz = 2 * kPi / (n[2] * dx[2]);
  return sin(kx * i * dx[0]) * cos(ky * j * dx[1]) * cos(kz * k * dx[2]);
}

/* projection of the x velocity on the mode */
static double amplitude(const int n[3], const double dx[3], const double* u) {
  double num = 0, den = 0;
  size_t p = 0;
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i, ++p) {
        const double m = mode(n, dx, i, j, k);
        num += u[p] * m;
        den += m * m;
      }
  return num / den;
}

int main(int argc, char** argv) {
  const int steps = argc > 1 ? atoi(argv[1]) : 300;
  const int storage = argc > 2 ? atoi(argv[2]) : RMRT_F32DEV;
  if (steps < 1 || storage < 0 || storage > 2) {
    fprintf(stderr, "usage: rmrt_demo [steps >= 1] [storage 0|1|2]\n");
    return 2;
  }

  rmrt_params p = {0};
  p.lattice = RMRT_Q19;
  p.equation = RMRT_NSE;
  p.storage = storage;
  p.pattern = RMRT_AA;
  p.n[0] = 48, p.n[1] = 40, p.n[2] = 24;
  p.dx[0] = 1.0, p.dx[1] = 1.0, p.dx[2] = 2.0;
  p.cs2 = 1.0 / 3.0;
  p.nu = 0.02;
  p.nu_b = -1.0; /* default bulk viscosity 2 nu / d */
  p.s_hi = -1.0; /* default: s_nu */
  p.w_corner = -1.0;
  p.rho0 = 1.0;

  const size_t N = (size_t)p.n[0] * p.n[1] * p.n[2];
  const double U0 = 1e-3;
  const double kx = 2 * kPi / (p.n[0] * p.dx[0]), ky = 2 * kPi / (p.n[1] * p.dx[1]),
               kz = 2 * kPi / (p.n[2] * p.dx[2]);

  /* divergence-free initial velocity, uniform density (host, then device) */
  double* rho_h = (double*)malloc(N * sizeof(double));
  double* u_h = (double*)malloc(3 * N * sizeof(double));
  if (!rho_h || !u_h) return 1;
  size_t q = 0;
  for (int k = 0; k < p.n[2]; ++k)
    for (int j = 0; j < p.n[1]; ++j)
      for (int i = 0; i < p.n[0]; ++i, ++q) {
        const double x = i * p.dx[0], y = j * p.dx[1], z = k * p.dx[2];
        rho_h[q] = 1.0;
        u_h[q] = U0 * sin(kx * x) * cos(ky * y) * cos(kz * z);
        u_h[N + q] = -U0 * (kx / ky) * cos(kx * x) * sin(ky * y) * cos(kz * z);
        u_h[2 * N + q] = 0.0;
      }

  size_t bytes = 0;
  RMRT_OK_OR_EXIT(rmrt_population_bytes(&p, &bytes));
  void *f = NULL, *rho_d = NULL, *u_d = NULL;
  HIP_OK(hipMalloc(&f, bytes)); /* caller-owned population buffer */
  HIP_OK(hipMalloc(&rho_d, N * sizeof(double)));
  HIP_OK(hipMalloc(&u_d, 3 * N * sizeof(double)));
  HIP_OK(hipMemcpy(rho_d, rho_h, N * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(u_d, u_h, 3 * N * sizeof(double), hipMemcpyHostToDevice));
  hipStream_t s;
  HIP_OK(hipStreamCreate(&s));

  rmrt_ctx* ctx = NULL;
  RMRT_OK_OR_EXIT(rmrt_init(&ctx, &p, f, NULL, NULL, (const double*)rho_d, (const double*)u_d, 1, s));
  double r0[4], r1[4];
  RMRT_OK_OR_EXIT(rmrt_reduce(ctx, r0, s));
  RMRT_OK_OR_EXIT(rmrt_moments(ctx, rho_d, u_d, RMRT_OUT_F64, s));
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipMemcpy(u_h, u_d, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
  const double a0 = amplitude(p.n, p.dx, u_h);

  RMRT_OK_OR_EXIT(rmrt_step(ctx, steps, s));
  RMRT_OK_OR_EXIT(rmrt_reduce(ctx, r1, s));
  RMRT_OK_OR_EXIT(rmrt_moments(ctx, rho_d, u_d, RMRT_OUT_F64, s));
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipMemcpy(u_h, u_d, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
  const double a1 = amplitude(p.n, p.dx, u_h);

  printf("steps %d\nstorage %d\nnodes %zu\n", steps, storage, N);
  printf("mass0 %.17g\nmass1 %.17g\n", r0[0], r1[0]);
  printf("mom1_x %.17g\nmom1_y %.17g\nmom1_z %.17g\n", r1[1], r1[2], r1[3]);
  printf("amp0 %.17g\namp1 %.17g\n", a0, a1);
  printf("nu %.17g\nnu_fit %.17g\n", p.nu, -log(a1 / a0) / (steps * (kx * kx + ky * ky + kz * kz)));

  RMRT_OK_OR_EXIT(rmrt_free(ctx));
  HIP_OK(hipStreamDestroy(s));
  HIP_OK(hipFree(f));
  HIP_OK(hipFree(rho_d));
  HIP_OK(hipFree(u_d));
  free(rho_h);
  free(u_h);
  return 0;
}
