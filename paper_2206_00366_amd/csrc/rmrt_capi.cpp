// Host side of the C ABI declared in include/rmrt.h: parameter derivation and
// validation, coefficient tables, contexts, graph-captured stepping, FP64
// reductions and the batched persistent path with its autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rmrt.h"
#include "lbm_kernels.hpp"

using namespace rmrt;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                            \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(RMRT_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// The two timing events of the tuners, destroyed on every return path.
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// ---------------------------------------------------------------------------
// Lattice and parameter derivation (Sec. III, Sec. IV, Sec. V)
// ---------------------------------------------------------------------------
struct Derived {
  int lattice, q, d;
  double c[3], cs2, dt, r[3];
  double w[27];
  double nu, nu_b, s_nu, s_s[3], s_b[3], s_hi;
  double nu_diag[3], nu_pair[3], nu_b_ax[3];  // viscosity tensor entries (eq. 4-29)
  double s_pair[3];   // off-diagonal rates (xy, xz, yz)
  int hl;             // He-Luo equilibrium
  double Sbar[3][3];  // second-order diagonal block (eq. 5-8-1)
  double D0, D2;
  int e[27][3];
};

int lattice_q(int lat) {
  switch (lat) {
    case RMRT_Q9: return 9;
    case RMRT_Q19: return 19;
    case RMRT_Q27: return 27;
    case RMRT_Q5: return 5;
    default: return 7;
  }
}
bool lattice_2d(int lat) { return lat == RMRT_Q9 || lat == RMRT_Q5; }

size_t elem_size(int storage) { return storage == RMRT_F64 ? 8 : (storage == RMRT_F32DEV ? 4 : 2); }

// Stream stride (in elements) of the population layout for N nodes: stream j
// occupies elements [j ld, j ld + N) of a population buffer.  Measured on
// MI355X (rD3Q19 FP32, cap 3): with ld = N, 256 x 256 x 127 and 200 x 160 x 260
// run at 4.6 TB/s against 5.6 TB/s at 256 x 256 x 128; a stream stride of
// 31.75 MiB (64 KiB-aligned) is as slow, strides that are whole MiB run at
// 5.3-5.6 TB/s.  Streams of 16 MiB and more are therefore padded to whole MiB,
// streams of 1-16 MiB to 64 KiB (the 64-domain rD3Q27 batch: 4.6 -> 5.0 TB/s),
// smaller ones to 4 KiB; the padding costs at most 1/16 of the buffer beyond
// 1 MiB per stream.
uint32_t stream_ld(uint32_t N, int storage) {
  const uint64_t es = elem_size(storage);
  const uint64_t bytes = (uint64_t)N * es;
  const uint64_t align = bytes >= (16u << 20) ? (1u << 20) : (bytes >= (1u << 20) ? (64u << 10) : 4096u);
  return (uint32_t)((bytes + align - 1) / align * align / es);
}
bool lattice_linear(int lat) { return lat == RMRT_Q5 || lat == RMRT_Q7; }

// Do the rows of the population streams straddle 128-byte cache lines?  Then
// the odd AA step's neighbour offsets along y (and z) are not whole lines and
// its accesses share lines between neighbouring tiles.
bool rows_straddle_lines(const rmrt_params& p) {
  return ((uint64_t)p.n[0] * elem_size(p.storage)) % 128u != 0;
}

bool bhll_relaxation(const Derived& v, double rb[6][6]);

int derive(const rmrt_params* p, Derived& v) {
  if (!p) return fail(RMRT_EINVAL, "params is NULL");
  if (p->lattice < RMRT_Q9 || p->lattice > RMRT_Q7) return fail(RMRT_EINVAL, "unknown lattice %d", p->lattice);
  if (p->equation != RMRT_NSE && p->equation != RMRT_NCDE)
    return fail(RMRT_EINVAL, "unknown equation %d", p->equation);
  if (p->storage < RMRT_F64 || p->storage > RMRT_F16DEV) return fail(RMRT_EINVAL, "unknown storage %d", p->storage);
  if (p->pattern != RMRT_AB && p->pattern != RMRT_AA) return fail(RMRT_EINVAL, "unknown pattern %d", p->pattern);
  v.lattice = p->lattice;
  v.q = lattice_q(p->lattice);
  v.d = lattice_2d(p->lattice) ? 2 : 3;
  if (lattice_linear(p->lattice) && p->equation != RMRT_NCDE)
    return fail(RMRT_EINVAL, "rD2Q5 / rD3Q7 carry the NCDE only (linear equilibrium, eq. 4-16)");
  for (int a = 0; a < 3; ++a)
    if (p->n[a] < 1) return fail(RMRT_EINVAL, "n[%d] = %d < 1", a, p->n[a]);
  if (v.d == 2 && p->n[2] != 1) return fail(RMRT_EINVAL, "2D lattices need n[2] == 1");
  const double N = (double)p->n[0] * p->n[1] * p->n[2];
  if (N * v.q >= 4294967295.0) return fail(RMRT_EUNSUPPORTED, "q * N must be below 2^32");
  if ((double)stream_ld((uint32_t)N, p->storage) * v.q >= 4294967295.0)
    return fail(RMRT_EUNSUPPORTED, "q * stream stride must be below 2^32");
  v.dt = p->dt > 0 ? p->dt : 1.0;
  for (int a = 0; a < 3; ++a) {
    double dx = (a < v.d) ? p->dx[a] : 1.0;
    if (!(dx > 0)) return fail(RMRT_EINVAL, "dx[%d] must be > 0", a);
    v.c[a] = dx / v.dt;  // c_a = dx_a / dt (Sec. III)
  }
  double cmin2 = v.c[0] * v.c[0];
  for (int a = 1; a < v.d; ++a) cmin2 = std::min(cmin2, v.c[a] * v.c[a]);
  v.cs2 = p->cs2 > 0 ? p->cs2 : cmin2 / 3.0;
  for (int a = 0; a < 3; ++a) {
    v.r[a] = v.cs2 / (v.c[a] * v.c[a]);
    if (a < v.d && !(v.r[a] > 0 && v.r[a] < 1))
      return fail(RMRT_EINVAL, "need 0 < cs2 / c_%d^2 < 1 (got %g)", a, v.r[a]);
  }
  for (int j = 0; j < 27; ++j)
    for (int a = 0; a < 3; ++a) v.e[j][a] = (v.d == 2) ? (j < 9 ? kE9[j][a] : 0) : kE27[j][a];
  // weights: eq. 3-3-5 (rD2Q9), eq. 3-3-8 (rD3Q27; omega_19 = 0 gives rD3Q19),
  // Remark I of Sec. III (rD2Q5, rD3Q7: omega_a = r_a / 2 on the axes)
  std::fill(v.w, v.w + 27, 0.0);
  const double* r = v.r;
  if (lattice_linear(p->lattice)) {
    for (int a = 0; a < v.d; ++a) v.w[1 + a] = v.w[1 + v.d + a] = r[a] / 2.0;
  } else if (p->lattice == RMRT_Q9) {
    const double w5 = r[0] * r[1] / 4.0;
    const double w1 = r[0] / 2.0 - 2.0 * w5, w2 = r[1] / 2.0 - 2.0 * w5;
    const double ws[9] = {0, w1, w2, w1, w2, w5, w5, w5, w5};
    for (int j = 1; j < 9; ++j) v.w[j] = ws[j];
  } else {
    double w19 = 0.0;
    if (p->lattice == RMRT_Q27) w19 = p->w_corner >= 0 ? p->w_corner : r[0] * r[1] * r[2] / 8.0;
    const double w7 = r[0] * r[1] / 4.0 - 2.0 * w19;
    const double w11 = r[0] * r[2] / 4.0 - 2.0 * w19;
    const double w15 = r[1] * r[2] / 4.0 - 2.0 * w19;
    const double w1 = r[0] / 2.0 - 2.0 * (w7 + w11) - 4.0 * w19;
    const double w2 = r[1] / 2.0 - 2.0 * (w7 + w15) - 4.0 * w19;
    const double w3 = r[2] / 2.0 - 2.0 * (w11 + w15) - 4.0 * w19;
    const double base[7] = {0, w1, w2, w3, w1, w2, w3};
    for (int j = 1; j < 7; ++j) v.w[j] = base[j];
    for (int j = 7; j < 11; ++j) v.w[j] = w7;
    for (int j = 11; j < 15; ++j) v.w[j] = w11;
    for (int j = 15; j < 19; ++j) v.w[j] = w15;
    for (int j = 19; j < v.q; ++j) v.w[j] = w19;
  }
  double sum = 0;
  for (int j = 1; j < v.q; ++j) sum += v.w[j];
  v.w[0] = 1.0 - sum;
  if (std::fabs(v.w[0]) < 1e-14) v.w[0] = 0.0;   // rounding of an exact zero (e.g. rD3Q7, c_s^2 = c^2 / 3)
  for (int j = 0; j < v.q; ++j)
    if (!(v.w[j] >= 0)) return fail(RMRT_EINVAL, "weight w_%d = %g is negative", j, v.w[j]);
  if (p->storage == RMRT_F16DEV)
    for (int j = 0; j < v.q; ++j)
      if (!(v.w[j] > 0))
        return fail(RMRT_EINVAL, "FP16 deviation storage divides by the weights: w_%d = 0", j);

  v.D0 = p->D0;
  v.D2 = p->D2;
  v.hl = p->incompressible != 0;
  for (int k = 0; k < 3; ++k) v.nu_diag[k] = v.nu_pair[k] = v.nu_b_ax[k] = 0.0, v.s_pair[k] = 1.0;
  if (v.hl && !(p->rho0 > 0)) return fail(RMRT_EINVAL, "the He-Luo equilibrium needs rho0 > 0");
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) v.Sbar[a][b] = 0.0;
  if (p->equation == RMRT_NSE) {
    v.nu = p->nu;
    if (!(v.nu > 0)) return fail(RMRT_EINVAL, "nu must be > 0");
    v.nu_b = p->nu_b < 0 ? 2.0 * v.nu / v.d : p->nu_b;
    if (!(v.nu_b > 0)) return fail(RMRT_EINVAL, "nu_b must be > 0");
    // viscosity tensor entries of eq. 4-29 (diagonal xx, yy, zz; pairs xy,
    // xz, yz; bulk per axis); unset entries are isotropic
    for (int k = 0; k < 6; ++k)
      if (std::isnan(p->nu_tensor[k]) || (k < 3 && std::isnan(p->nu_b_axis[k])))
        return fail(RMRT_EINVAL, "viscosity tensor entry %d is NaN", k);
    for (int k = 0; k < 3; ++k) {
      v.nu_diag[k] = p->nu_tensor[k] > 0 ? p->nu_tensor[k] : v.nu;
      v.nu_pair[k] = p->nu_tensor[3 + k] > 0 ? p->nu_tensor[3 + k] : v.nu;
      v.nu_b_ax[k] = p->nu_b_axis[k] > 0 ? p->nu_b_axis[k] : v.nu_b;
    }
    // eq. 4-31 solved for the rates, entry by entry
    v.s_nu = 1.0 / (0.5 + v.nu / (v.cs2 * v.dt));
    for (int k = 0; k < 3; ++k) {
      v.s_pair[k] = 1.0 / (0.5 + v.nu_pair[k] / (v.cs2 * v.dt));
      if (!(v.s_pair[k] > 0 && v.s_pair[k] < 2)) return fail(RMRT_EINVAL, "s_ab = %g outside (0, 2)", v.s_pair[k]);
    }
    double a[3], b[3], Adiag[3];
    for (int k = 0; k < v.d; ++k) {
      const double g = v.c[k] * v.c[k] - v.cs2;
      v.s_s[k] = 1.0 / (0.5 + 2.0 * v.nu_diag[k] / (g * v.dt));
      v.s_b[k] = 1.0 / (0.5 + v.d * v.nu_b_ax[k] / (g * v.dt));
      a[k] = (1.0 / v.s_b[k] - 1.0 / v.s_s[k]) * g;
      b[k] = 1.0 / g;
      Adiag[k] = v.s_s[k];
    }
    // Sherman-Morrison form of the inverse of diag(1/s_s) + a b^T / d (eq. 5-8-1)
    double bAa = 0.0;
    for (int k = 0; k < v.d; ++k) bAa += b[k] * Adiag[k] * a[k] / v.d;
    for (int i = 0; i < v.d; ++i)
      for (int k = 0; k < v.d; ++k)
        v.Sbar[i][k] = (i == k ? Adiag[i] : 0.0) - Adiag[i] * (a[i] / v.d) * b[k] * Adiag[k] / (1.0 + bAa);
    v.s_hi = p->s_hi > 0 ? p->s_hi : v.s_nu;
    if (!(v.s_nu > 0 && v.s_nu < 2)) return fail(RMRT_EINVAL, "s_nu = %g outside (0, 2)", v.s_nu);
    for (int k = 0; k < v.d; ++k)
      if (!(v.s_s[k] > 0 && v.s_s[k] < 2 && v.s_b[k] > 0 && v.s_b[k] < 2))
        return fail(RMRT_EINVAL, "second-order rates outside (0, 2)");
  } else {
    v.nu = v.nu_b = 0.0;
    if (p->incompressible) return fail(RMRT_EINVAL, "the He-Luo equilibrium is an NSE option");
  }
  if (p->equation == RMRT_NSE && p->gamma0) return fail(RMRT_EINVAL, "gamma = 0 is an NCDE option (eq. 2-1)");
  if (p->equation == RMRT_NSE && p->c_zero) return fail(RMRT_EINVAL, "the C = 0 form is an NCDE option (eq. 4-16)");
  if (p->c_zero && p->diffusive) return fail(RMRT_EINVAL, "c_zero and diffusive are different NCDE models");
  if (p->central) {
    if (p->equation != RMRT_NSE) return fail(RMRT_EINVAL, "the central-moment collision is an NSE option");
    if (p->lattice != RMRT_Q9 && p->lattice != RMRT_Q27)
      return fail(RMRT_EUNSUPPORTED, "the central-moment collision is built for rD2Q9 and rD3Q27 (moment sets "
                                     "closed under the shift)");
  }
  if (p->hermite && p->equation != RMRT_NSE)
    return fail(RMRT_EINVAL, "the Hermite-moment collision is an NSE option");
  if (p->bhll) {
    if (p->equation != RMRT_NSE) return fail(RMRT_EINVAL, "the BHLL-moment collision is an NSE option");
    if (p->central || p->hermite)
      return fail(RMRT_EINVAL, "the BHLL basis is not combined with the central or Hermite one");
    if (p->lattice != RMRT_Q9)
      return fail(RMRT_EUNSUPPORTED, "the BHLL-moment collision is built for rD2Q9 (the basis of eq. Md2q9-3)");
  }
  if (p->equation == RMRT_NSE && p->diffusive) return fail(RMRT_EINVAL, "the diffusive scaling is an NCDE option");
  if (p->equation != RMRT_NSE) {
    if (!(p->D0 > 0)) return fail(RMRT_EINVAL, "D0 must be > 0 for the NCDE");
    if (p->D2 < 0) return fail(RMRT_EINVAL, "D2 must be >= 0");
    v.s_nu = 1.0;
    v.s_hi = p->s_hi > 0 ? p->s_hi : 1.0;
    for (int k = 0; k < 3; ++k) v.s_s[k] = v.s_b[k] = 1.0;
  }
  if (!(v.s_hi > 0 && v.s_hi < 2)) return fail(RMRT_EINVAL, "s_hi = %g outside (0, 2)", v.s_hi);
  if (p->bhll) {
    double rb[6][6];
    if (!bhll_relaxation(v, rb)) return fail(RMRT_EINVAL, "the BHLL basis matrix is singular");
  }
  return RMRT_OK;
}

// L(k) = sum_j w_j prod_a c_ja^k_a (brute force over the lattice)
double lattice_sum(const Derived& v, const int k[3]) {
  double s = 0.0;
  for (int j = 0; j < v.q; ++j) {
    double t = v.w[j];
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < k[a]; ++i) t *= v.e[j][a] * v.c[a];
    s += t;
  }
  return s;
}

void invert3(const double A[3][3], double B[3][3], int d) {
  // Gauss-Jordan on the leading d x d block; remaining diagonal set to 1
  double M[3][6];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 6; ++j) M[i][j] = 0.0;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) M[i][j] = (i < d && j < d) ? A[i][j] : (i == j ? 1.0 : 0.0);
    M[i][3 + i] = 1.0;
  }
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
    for (int j = 0; j < 6; ++j) std::swap(M[c][j], M[piv][j]);
    const double inv = 1.0 / M[c][c];
    for (int j = 0; j < 6; ++j) M[c][j] *= inv;
    for (int r = 0; r < 3; ++r)
      if (r != c) {
        const double f = M[r][c];
        for (int j = 0; j < 6; ++j) M[r][j] -= f * M[c][j];
      }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[i][j] = M[i][3 + j];
}

// In-place inverse of the n x n row-major matrix A (Gauss-Jordan with partial
// pivoting); false when a pivot vanishes.
bool invert_small(double* A, int n) {
  if (n < 1 || n > 9) return false;
  double inv[81];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i * n + j] = i == j ? 1.0 : 0.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
    if (!(std::fabs(A[piv * n + col]) > 0)) return false;
    for (int j = 0; j < n; ++j) {
      std::swap(A[col * n + j], A[piv * n + j]);
      std::swap(inv[col * n + j], inv[piv * n + j]);
    }
    const double d = 1.0 / A[col * n + col];
    for (int j = 0; j < n; ++j) {
      A[col * n + j] *= d;
      inv[col * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = A[r * n + col];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[r * n + j] -= f * A[col * n + j];
        inv[r * n + j] -= f * inv[col * n + j];
      }
    }
  }
  std::copy(inv, inv + n * n, A);
  return true;
}

// The BHLL-moment relaxation (Sec. V, eq. Md2q9-2 / Md2q9-3, with eq. 5-1-2)
// in the scaled raw basis of the kernels.  Rows and columns 0..8 below are the
// raw moments 1, x, y, x^2, y^2, xy, xy^2, x^2y, x^2y^2 of the printed matrix.
// N = N_BHLL(a) diag(c_x^-order) with a = c_y / c_x maps the raw moments to the
// BHLL ones; Sbar_B keeps the blocks of N S N^-1 between moments of one order
// (the second-order block of eq. 5-8 carried over by similarity, s_xy on p_xy,
// s_hi on q_x, q_y and epsilon); the kernels apply D^-1 N^-1 Sbar_B N D with D =
// diag(c_x^i c_y^j) to the non-conserved tensor slots 2, 4, 5, 6, 7, 8.
bool bhll_relaxation(const Derived& v, double rb[6][6]) {
  static const int ex[9][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {0, 2}, {1, 1}, {1, 2}, {2, 1}, {2, 2}};
  const double a = v.c[1] / v.c[0], a2 = a * a;
  const double Nb[81] = {1, 0, 0, 0, 0, 0, 0, 0, 0,
                         0, 1, 0, 0, 0, 0, 0, 0, 0,
                         0, 0, 1, 0, 0, 0, 0, 0, 0,
                         -2 * a2 - 2, 0, 0, 3, 3, 0, 0, 0, 0,
                         -2 * a2 + 2, 0, 0, 3 * a2, -3 / a2, 0, 0, 0, 0,
                         0, 0, 0, 0, 0, 1, 0, 0, 0,
                         0, -2, 0, 0, 0, 0, 3 / a2, 0, 0,
                         0, 0, -2, 0, 0, 0, 0, 3, 0,
                         4, 0, 0, -6, -6 / a2, 0, 0, 0, 9 / a2};
  int ord[9];
  double N[81], Ni[81], S[81] = {0}, T[81], Sb[81], R[81];
  for (int i = 0; i < 9; ++i) ord[i] = ex[i][0] + ex[i][1];
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) N[i * 9 + j] = Nb[i * 9 + j] * std::pow(v.c[0], -ord[j]);
  std::copy(N, N + 81, Ni);
  if (!invert_small(Ni, 9)) return false;
  // the raw model's relaxation matrix (its conserved rows play no part)
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) S[(3 + i) * 9 + 3 + j] = v.Sbar[i][j];
  S[5 * 9 + 5] = v.s_pair[0];
  for (int i = 6; i < 9; ++i) S[i * 9 + i] = v.s_hi;
  auto mul = [](const double* X, const double* Y, double* Z) {
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 9; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 9; ++k) acc += X[i * 9 + k] * Y[k * 9 + j];
        Z[i * 9 + j] = acc;
      }
  };
  mul(N, S, T);
  mul(T, Ni, Sb);
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j)
      if (ord[i] != ord[j]) Sb[i * 9 + j] = 0.0;
  mul(Ni, Sb, T);
  mul(T, N, R);
  // tensor slot (i + 3 j) of raw row r; non-conserved slot k: 2, then 4 .. 8
  auto slot_k = [&](int r) {
    const int sl = ex[r][0] + 3 * ex[r][1];
    return sl == 2 ? 0 : sl - 3;
  };
  for (int r = 0; r < 9; ++r) {
    if (ord[r] < 2) continue;
    for (int s = 0; s < 9; ++s) {
      if (ord[s] < 2) continue;
      const double dr = std::pow(v.c[0], ex[r][0]) * std::pow(v.c[1], ex[r][1]);
      const double ds = std::pow(v.c[0], ex[s][0]) * std::pow(v.c[1], ex[s][1]);
      rb[slot_k(r)][slot_k(s)] = R[r * 9 + s] * ds / dr;
    }
  }
  return true;
}

template <typename T>
void fill_coef(const rmrt_params* p, const Derived& v, Coef<T>& C) {
  std::memset(&C, 0, sizeof(C));
  const double dt = v.dt;
  C.rho0 = (T)p->rho0;
  C.cs2 = (T)v.cs2;
  C.inv_cs2 = (T)(1.0 / v.cs2);
  C.dt = (T)dt;
  for (int a = 0; a < 3; ++a) {
    C.c[a] = (T)v.c[a];
    C.inv_c[a] = (T)(1.0 / v.c[a]);
  }
  for (int j = 0; j < 27; ++j) {
    C.w[j] = (T)v.w[j];
    C.iw[j] = v.w[j] > 0 ? (T)(1.0 / v.w[j]) : (T)0;
  }
  // by weight class (rest, x, y, z axes, xy, xz, yz edges, corners); all
  // velocities of a class share one weight
  for (int k = 0; k < 8; ++k) C.wc[k] = C.iwc[k] = (T)0;
  for (int j = 0; j < v.q; ++j) {
    const int x = v.e[j][0] != 0, y = v.e[j][1] != 0, z = v.e[j][2] != 0, n = x + y + z;
    const int k = n == 0 ? 0 : n == 3 ? 7 : n == 1 ? (x ? 1 : y ? 2 : 3) : (x && y ? 4 : x && z ? 5 : 6);
    C.wc[k] = C.w[j];
    C.iwc[k] = C.iw[j];
  }
  // scaled raw-moment tables of g_eq (eq. 3-3, 3-4) for every tensor slot
  const int d = v.d;
  const double cs2 = v.cs2;
  const int nslots = d == 2 ? 9 : 27;
  for (int n = 0; n < nslots; ++n) {
    const int ex[3] = {n % 3, (n / 3) % 3, n / 9};
    double scale = 1.0;
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < ex[a]; ++i) scale *= v.c[a];
    int odd[3], nodd = 0;
    for (int a = 0; a < 3; ++a)
      if (ex[a] & 1) odd[nodd++] = a;
    if (nodd == 0) {
      C.E0[n] = (T)(lattice_sum(v, ex) / scale);
      const double L0 = lattice_sum(v, ex);
      for (int a = 0; a < d; ++a) {
        int k[3] = {ex[0], ex[1], ex[2]};
        k[a] += 2;
        const double g = v.c[a] * v.c[a] - cs2;
        C.E2[n][a] = (T)((lattice_sum(v, k) - cs2 * L0) / (cs2 * g * scale));
      }
    } else if (nodd == 1) {
      int k[3] = {ex[0], ex[1], ex[2]};
      k[odd[0]] += 1;
      C.E1[n] = (T)(lattice_sum(v, k) / (cs2 * scale));
    } else if (nodd == 2) {
      int k[3] = {ex[0], ex[1], ex[2]};
      k[odd[0]] += 1;
      k[odd[1]] += 1;
      C.E3[n] = (T)(lattice_sum(v, k) / (cs2 * cs2 * scale));
    }
  }
  // relaxation: scaled diagonal block, off-diagonal and higher rates
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      C.Sd[a][b] = (a < d && b < d) ? (T)(v.Sbar[a][b] * v.c[b] * v.c[b] / (v.c[a] * v.c[a])) : (T)0;
      C.IhS[a][b] = (T)((a == b ? 1.0 : 0.0) - ((a < d && b < d) ? 0.5 * v.Sbar[a][b] : 0.0));
    }
  for (int k = 0; k < 3; ++k) {
    C.s_off[k] = (T)v.s_pair[k];
    C.ihs_off[k] = (T)(1.0 - 0.5 * v.s_pair[k]);
  }
  C.hl = v.hl ? 1u : 0u;
  C.s_hi = (T)v.s_hi;
  // source terms carry the factor dt (m* gets dt (m_G + (I - S/2) m_F))
  for (int a = 0; a < 3; ++a) {
    const double F = (a < d) ? p->force[a] : 0.0;
    C.force[a] = (T)(dt * F);
    C.half_force[a] = (T)(0.5 * dt * F);
    C.adv[a] = (T)((a < d) ? p->adv[a] : 0.0);
  }
  C.source = (T)(dt * p->source);
  // gamma = 0 form and diffusive scaling (NCDE): populations are f, phi = sum f,
  // no dt S / 2 shift (eq. 2-1 without the dt^2/2 D F term)
  const bool no_shift = p->equation == RMRT_NCDE && (p->gamma0 || p->diffusive);
  C.half_source = no_shift ? (T)0 : (T)(0.5 * dt * p->source);
  // C = 0 form (eq. 4-16: the reduced lattices, or the c_zero option): no
  // C = phi u u in the equilibrium, G from dB/dt with the history field
  const bool c0 = p->equation == RMRT_NCDE && (lattice_linear(p->lattice) || p->c_zero);
  for (int a = 0; a < 3; ++a) {
    const bool diff = p->equation == RMRT_NCDE && p->diffusive;
    C.adv_c[a] = (diff || c0) ? (T)0 : C.adv[a];   // eq. 4-17 and eq. 4-16: C = 0
    C.adv_g[a] = diff ? (T)0 : C.adv[a];           // eq. 4-17: G = 0
  }
  C.hist_g = c0 ? 1u : 0u;
  C.basis = (p->equation == RMRT_NSE && p->central ? BASIS_CENTRAL : 0u) |
            (p->equation == RMRT_NSE && p->hermite ? BASIS_HERMITE : 0u) |
            (p->equation == RMRT_NSE && p->bhll ? BASIS_BHLL : 0u);
  if (C.basis & BASIS_BHLL) {
    double rb[6][6] = {};
    bhll_relaxation(v, rb);   // derive() has checked that N is invertible
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) C.rb[i][j] = (T)rb[i][j];
  }
  for (int a = 0; a < 3; ++a) C.hth[a] = (T)(a < v.d ? v.cs2 / (v.c[a] * v.c[a]) : 0.0);
  // factors of the per-node source fields
  C.half_dt = (T)(0.5 * dt);
  C.dt_cs2 = (T)(dt * cs2);
  C.half_dt_cs2 = (T)(0.5 * dt * cs2);
  C.half_src_factor = no_shift ? (T)0 : (T)(0.5 * dt);
  C.cs2_source = (T)(dt * cs2 * p->source);
  C.half_cs2_source = (T)(0.5 * dt * cs2 * p->source);
  C.D0 = (T)p->D0;
  C.D2 = (T)p->D2;
  C.inv_cs2_dt = (T)(1.0 / (cs2 * dt));
  C.inv_dt = (T)(1.0 / dt);
}

uint32_t magic(uint32_t d) { return d <= 1 ? 0xffffffffu : (uint32_t)(0x100000000ull / d); }

void fill_domain(const rmrt_params* p, const Derived& v, DomainDev& D, void* fa, void* fb, const uint8_t* solid) {
  std::memset(&D, 0, sizeof(D));
  fill_coef<double>(p, v, D.cd);
  fill_coef<float>(p, v, D.cf);
  double IhS[3][3], K[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) IhS[a][b] = (a == b ? 1.0 : 0.0) - 0.5 * v.Sbar[a][b];
  invert3(IhS, K, v.d);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) D.ic.Kd[a][b] = (a < v.d && b < v.d) ? K[a][b] : 0.0;
  for (int k = 0; k < 3; ++k) D.ic.k_off[k] = 1.0 / (1.0 - 0.5 * v.s_pair[k]);
  D.ic.nu = v.nu;
  D.ic.nu_b = v.nu_b;
  for (int k = 0; k < 3; ++k) {
    D.ic.nu_diag[k] = v.nu_diag[k];
    D.ic.nu_pair[k] = v.nu_pair[k];
    D.ic.nu_b_ax[k] = v.nu_b_ax[k];
  }
  double den = 1.0;
  for (int k = 0; k < 3; ++k) {
    const bool axis = k < v.d, pair = (v.d == 3) || k == 0;
    D.ic.inv2nu_diag[k] = axis ? 0.5 / v.nu_diag[k] : 0.0;
    D.ic.bulk_excess[k] = axis ? v.nu_b_ax[k] - 2.0 * v.nu_diag[k] / v.d : 0.0;
    D.ic.inv2nu_pair[k] = pair ? 0.5 / v.nu_pair[k] : 0.0;
    den += D.ic.bulk_excess[k] * D.ic.inv2nu_diag[k];
  }
  D.ic.inv_trace_den = 1.0 / den;
  D.nx = p->n[0];
  D.ny = p->n[1];
  D.nz = p->n[2];
  D.nxny = D.nx * D.ny;
  D.N = D.nxny * D.nz;
  D.ld = stream_ld(D.N, p->storage);
  D.mnx = magic(D.nx);
  D.mnxny = magic(D.nxny);
  D.walls = p->wall_faces & 63u;
  if (v.d == 2) D.walls &= 15u;
  D.has_solid = solid != nullptr;
  D.lattice = p->lattice;
  D.equation = p->equation;
  D.storage = p->storage;
  D.fa = fa;
  D.fb = fb;
  D.solid = solid;
  D.oob_limit = D.N;
  D.oob = nullptr;
}

bool c_zero_form(const rmrt_params* p) {
  return p->equation == RMRT_NCDE && (lattice_linear(p->lattice) || p->c_zero);
}

bool has_force(const rmrt_params* p) {
  if (p->source != 0.0) return true;
  if (c_zero_form(p))   // the dB/dt term G of eq. 4-16
    for (int a = 0; a < 3; ++a)
      if (p->adv[a] != 0.0) return true;
  if (p->equation == RMRT_NSE)
    for (int a = 0; a < 3; ++a)
      if (p->force[a] != 0.0) return true;
  return false;
}


// ---------------------------------------------------------------------------
// Dispatch onto the per-(lattice, storage) instantiations
// ---------------------------------------------------------------------------
template <template <int, int> class>
struct Unused {};

#define RMRT_DISPATCH(FN, lat, st, arg)                                               \
  do {                                                                                \
    switch ((lat) * 3 + (st)) {                                                       \
      case 0: return FN<LAT_Q9, ST_F64>(arg);                                         \
      case 1: return FN<LAT_Q9, ST_F32>(arg);                                         \
      case 2: return FN<LAT_Q9, ST_F16>(arg);                                         \
      case 3: return FN<LAT_Q19, ST_F64>(arg);                                        \
      case 4: return FN<LAT_Q19, ST_F32>(arg);                                        \
      case 5: return FN<LAT_Q19, ST_F16>(arg);                                        \
      case 6: return FN<LAT_Q27, ST_F64>(arg);                                        \
      case 7: return FN<LAT_Q27, ST_F32>(arg);                                        \
      case 8: return FN<LAT_Q27, ST_F16>(arg);                                        \
      case 9: return FN<LAT_Q5, ST_F64>(arg);                                         \
      case 10: return FN<LAT_Q5, ST_F32>(arg);                                        \
      case 11: return FN<LAT_Q5, ST_F16>(arg);                                        \
      case 12: return FN<LAT_Q7, ST_F64>(arg);                                        \
      case 13: return FN<LAT_Q7, ST_F32>(arg);                                        \
      case 14: return FN<LAT_Q7, ST_F16>(arg);                                        \
    }                                                                                 \
    return hipErrorInvalidValue;                                                      \
  } while (0)

hipError_t dispatch_step(int lat, int st, const StepLaunch& a) { RMRT_DISPATCH(launch_step, lat, st, a); }
hipError_t dispatch_init(int lat, int st, const AuxLaunch& a) { RMRT_DISPATCH(launch_init, lat, st, a); }
hipError_t dispatch_moments(int lat, int st, const AuxLaunch& a) { RMRT_DISPATCH(launch_moments, lat, st, a); }
hipError_t dispatch_populations(int lat, int st, const AuxLaunch& a) {
  RMRT_DISPATCH(launch_populations, lat, st, a);
}
hipError_t dispatch_reduce(int lat, int st, const AuxLaunch& a) { RMRT_DISPATCH(launch_reduce, lat, st, a); }
hipError_t dispatch_residual(int lat, int st, const AuxLaunch& a) { RMRT_DISPATCH(launch_residual, lat, st, a); }
hipError_t dispatch_local(int lat, int st, const AuxLaunch& a) { RMRT_DISPATCH(launch_local, lat, st, a); }
hipError_t dispatch_links(int lat, const DomainDev* doms, uint32_t dom, void* out, unsigned grid, hipStream_t s) {
  switch (lat) {
    case LAT_Q9: return launch_links<LAT_Q9>(doms, dom, out, grid, s);
    case LAT_Q19: return launch_links<LAT_Q19>(doms, dom, out, grid, s);
    case LAT_Q27: return launch_links<LAT_Q27>(doms, dom, out, grid, s);
    case LAT_Q5: return launch_links<LAT_Q5>(doms, dom, out, grid, s);
    case LAT_Q7: return launch_links<LAT_Q7>(doms, dom, out, grid, s);
  }
  return hipErrorInvalidValue;
}

constexpr unsigned kAuxBlock = 256;
// Launch shape of the single-domain step.  Measured on MI355X: one workgroup
// per 256-node tile with hardware scheduling beats persistent grids (whose
// tile loop serialises loads behind the previous tile's stores).  For the 3D
// lattices with 4- and 8-byte storage a cap of 3-4 resident workgroups per CU
// (12-16 waves) beats full occupancy (rD3Q19 FP32 forward order: 5.2 -> 5.65
// TB/s): fewer waves issuing q concurrent address streams keep HBM rows open
// longer.  FP16 storage and the 2D lattices prefer no cap, rD2Q9 and rD2Q5 the
// XCD-contiguous tile order.
constexpr int kDefaultBlocksPerCU = 0;
constexpr uint32_t kDefaultFlags = 0u;
void default_launch(const rmrt_params& p, bool bounded, int& blocks_per_cu, uint32_t& flags) {
  blocks_per_cu = 0;
  // Buffer addressing everywhere it applies (graph replay at 256 x 256 x 128
  // or 2048 x 1024: rD3Q19 FP32 5.58 -> 5.73 TB/s, FP16 5.03 -> 5.31, rD3Q27
  // FP32 5.30 -> 5.45, FP16 4.49 -> 4.85, the others equal or better).  The
  // reduced lattices have only 5 or 7 loads per node and want every wave they
  // can get (rD3Q7 FP32: 7.0 TB/s uncapped, 6.1 with a cap of 3).
  // Alternating tile order everywhere: each step starts on the tiles the
  // previous one ended with, still held by the MALL and the L2 (rD3Q19 FP32
  // 5.74 -> 6.45 TB/s of algorithmic traffic, FP16 +11%, rD3Q27 +10%; the
  // MALL-resident 2048 x 1024 rD2Q9 / rD2Q5 FP32 cases +14% / +20%).
  flags = STEP_BUFFER_OFFSETS | STEP_ALTERNATE_ORDER;
  // XCD chunks wherever rows straddle cache lines and the tiles are not
  // already contiguous per XCD (500-1000-step graph replays, plain / chunked,
  // us per step): rD3Q27 FP32 200 x 160 x 260 periodic 314.0 / 304.6, 223 x
  // 116 x 100 periodic 98.9 / 91.7, with walls 102.5 / 95.3; rD3Q19 FP16
  // 250 x 256 x 128 125.4 / 110.6, FP64 446.7 / 435.3, FP32 207.3 / 209.3,
  // FP32 223 x 116 x 100 with walls and force 66.0 / 62.0.  Rows of whole
  // lines (256 x 256 x 128) lose with them (rD3Q19 FP32 199.2 / 224.3).
  if (rows_straddle_lines(p) && p.lattice != RMRT_Q9 && p.lattice != RMRT_Q5 &&
      !(p.lattice == RMRT_Q7 && p.storage != RMRT_F64))
    flags |= STEP_XCD_CHUNKS;
  if (p.lattice == RMRT_Q9 || p.lattice == RMRT_Q5) {
    flags |= STEP_XCD_ORDER;
  } else if (p.lattice == RMRT_Q7) {
    if (p.storage == RMRT_F64)
      blocks_per_cu = 3;
    else
      flags |= STEP_XCD_ORDER;
  } else if (p.storage == RMRT_F32DEV) {
    // Residency caps, 500-step graph replays on two MI355X (us per step, cap
    // 3 / 4): rD3Q19 256 x 256 x 128 periodic 195.6 / 190.1 (the odd phase
    // gains 5%), 256 x 128 x 128 with walls and force 118.3 / 104.6; rD3Q27
    // periodic 291.7 / 297.5 (cap 2 ties cap 3), 223 x 116 x 100 and
    // 144^3 with walls and force 106.6 / 103.4 and 121.3 / 115.4.
    blocks_per_cu = (p.lattice == RMRT_Q19 || bounded || has_force(&p)) ? 4 : 3;
  } else if (p.storage == RMRT_F64) {
    blocks_per_cu = 3;   // rD3Q19 / rD3Q27 FP64: 440 / 642 us at caps 2 and 3, 460 / 667 at 4
  }
}
constexpr uint32_t kLdsPerCU = 160u * 1024u;  // gfx950 LDS per compute unit
constexpr unsigned kMaxAuxGrid = 2048;

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the allocation-free reduction (rmrt_reduce_noalloc): the block
// partial sums of k_reduce (5 doubles per workgroup, at most kMaxAuxGrid
// workgroups: 80 KiB per GPU, held until the process ends).  Host code never
// passes `scratch` itself to a kernel (in host code it names a host-side
// stand-in); it passes the device address that hipGetSymbolAddress returns
// for the GPU, looked up once per device at context creation with that device
// current.
// ---------------------------------------------------------------------------
namespace {
constexpr uint32_t kNoAllocBlocks = kMaxAuxGrid;
constexpr size_t kNoAllocDoubles = (size_t)kNoAllocBlocks * 5;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device), looked up on
// the first call for that device and cached.
int noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(RMRT_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return fail(RMRT_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(g_scratch_err[dev]));
    }
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return RMRT_OK;
}
static_assert(kMaxAuxGrid <= kNoAllocBlocks, "the reduction grid must fit the scratch");
}  // namespace

// shared error channel for the surrogate kernels' ABI (nn_capi.cpp)
int rmrt_set_error_(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

// ---------------------------------------------------------------------------
// Contexts
// ---------------------------------------------------------------------------
struct rmrt_ctx {
  rmrt_params p;
  Derived v;
  DomainDev hdom;
  DomainDev* ddoms = nullptr;  // device array holding this domain at index dom
  uint32_t dom = 0;
  bool owns_ddoms = false;
  rmrt_batch* batch = nullptr;
  long long steps = 0;
  double* partials = nullptr;  // kMaxAuxGrid x 5
  double* dres = nullptr;      // 8 doubles
  double* hres = nullptr;      // pinned, 8 doubles
  double* uprev = nullptr;
  bool have_prev = false;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  hipStream_t cap = nullptr;   // capture stream
  int cus = 256;               // compute units of the device
  void* links = nullptr;       // per-node link bits (solid-mask boundary mode)
  void* hist = nullptr;        // rD2Q5 / rD3Q7: previous-step phi per node (library-owned)
  int step_bc = 0;             // 0 periodic, 1 walls from coordinates, 2 link bits
  int blocks_per_cu = kDefaultBlocksPerCU;  // resident workgroups per CU (0: hardware limit)
  uint32_t flags = kDefaultFlags;
  int device = 0;              // the device current at creation
  void* sprev = nullptr;       // gamma = 0 NCDE with source fields: the previous step's source (library-owned)
  uint32_t* oob = nullptr;     // checked builds: the counter of neighbour indices out of range
};

namespace {

unsigned aux_grid(uint32_t N) {
  unsigned g = (N + kAuxBlock - 1) / kAuxBlock;
  return std::max(1u, std::min(g, kMaxAuxGrid));
}

// grid of a step launch: one block per tile, or (STEP_PERSISTENT) a persistent
// grid of cus * blocks_per_cu workgroups (a multiple of 8 when XCD-ordered)
// dynamic LDS that caps a non-persistent launch at blocks_per_cu resident workgroups per CU
uint32_t residency_lds(int blocks_per_cu, uint32_t flags) {
  if (blocks_per_cu <= 0 || (flags & STEP_PERSISTENT)) return 0;
  return (kLdsPerCU / (uint32_t)blocks_per_cu) & ~255u;
}

unsigned persistent_grid(uint32_t ntiles, int cus, int blocks_per_cu, uint32_t flags) {
  if (blocks_per_cu <= 0 || !(flags & STEP_PERSISTENT)) return ntiles;
  uint32_t g = (uint32_t)cus * (uint32_t)blocks_per_cu;
  if (flags & STEP_XCD_ORDER) g &= ~7u;
  if (g < 8) g = 8;
  return g >= ntiles ? ntiles : g;
}

int device_cus() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    return prop.multiProcessorCount;
  return 256;
}

AuxLaunch aux_of(const rmrt_ctx* c, hipStream_t s) {
  AuxLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.doms = c->ddoms;
  a.dom = c->dom;
  a.parity = (uint32_t)(c->steps & 1);
  a.ab = c->p.pattern == RMRT_AB;
  a.eq = c->p.equation;
  a.bc = (c->hdom.walls != 0 || c->hdom.has_solid) ? 1 : 0;
  a.swapped = (c->p.pattern == RMRT_AA) && (c->steps & 1);
  a.grid = aux_grid(c->hdom.N);
  a.block = kAuxBlock;
  a.stream = s;
  return a;
}

int ctx_alloc_scratch(rmrt_ctx* c) {
  HIP_TRY(hipMalloc(&c->partials, sizeof(double) * kMaxAuxGrid * 5));
  HIP_TRY(hipMalloc(&c->dres, sizeof(double) * 8));
  HIP_TRY(hipHostMalloc(&c->hres, sizeof(double) * 8, hipHostMallocDefault));
  return RMRT_OK;
}

// Destroy cached graph executables.  A graph launched by an earlier call may
// still run on some stream, so the device is drained first (graphs are dropped
// only on a launch-shape change, a cache eviction or a release).
template <class Map>
void drop_graphs(Map& graphs) {
  if (graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
}

// Release paths ignore the runtime's return codes: there is nothing left to
// recover and the first error has already been reported.
void ctx_release(rmrt_ctx* c) {
  (void)hipDeviceSynchronize();  // work issued on any stream may still use the buffers
  drop_graphs(c->graphs);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->partials) (void)hipFree(c->partials);
  if (c->dres) (void)hipFree(c->dres);
  if (c->hres) (void)hipHostFree(c->hres);
  if (c->uprev) (void)hipFree(c->uprev);
  if (c->links) (void)hipFree(c->links);
  if (c->hist) (void)hipFree(c->hist);
  if (c->sprev) (void)hipFree(c->sprev);
  if (c->oob) (void)hipFree(c->oob);
  if (c->owns_ddoms && c->ddoms) (void)hipFree(c->ddoms);
}

// Allocate the link bits of a context (hdom.links set); the caller uploads
// the parameter block and then runs build_links.
int alloc_links(rmrt_ctx* c) {
  const size_t w = lattice_q(c->p.lattice) <= 15 ? 2 : 4;
  HIP_TRY(hipMalloc(&c->links, w * c->hdom.N));
  c->hdom.links = c->links;
  c->step_bc = 2;
  return RMRT_OK;
}

int build_links(rmrt_ctx* c, hipStream_t s) {
  hipError_t e = dispatch_links(c->p.lattice, c->ddoms, c->dom, c->links, aux_grid(c->hdom.N), s);
  if (e != hipSuccess) return fail(RMRT_EHIP, "links launch: %s", hipGetErrorString(e));
  return RMRT_OK;
}

int launch_init_fields(rmrt_ctx* c, const double* rho, const double* u, int with_fne, hipStream_t s) {
  if (with_fne && c->p.equation != RMRT_NSE) return fail(RMRT_EUNSUPPORTED, "with_fne is NSE only");
  AuxLaunch a = aux_of(c, s);
  a.in0 = rho;
  a.in1 = u;
  a.flag = with_fne;
  hipError_t e = dispatch_init(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "init launch failed: %s", hipGetErrorString(e));
  c->have_prev = false;
  return RMRT_OK;
}

// Equation and source mode of a context's step kernel.
int step_eq(const rmrt_ctx* c) {
  if (c->p.equation == RMRT_NCDE && c->p.c_zero && !lattice_linear(c->p.lattice)) return EQ_NCDE_C0;
  if (c->p.equation == RMRT_NSE && (c->p.central || c->p.hermite || c->p.bhll)) return EQ_NSE_BASIS;
  return c->p.equation;
}
int step_force(const rmrt_ctx* c) {
  if (c->hdom.src_field) return F_FIELD;
  return has_force(&c->p) ? F_CONST : F_NONE;
}

// Buffer addressing takes 32-bit byte offsets: it serves domains whose
// population buffer is below 4 GiB.  Elsewhere the flag is a no-op.
bool buffer_offsets_apply(const rmrt_ctx* c) {
  const uint64_t bytes = (uint64_t)lattice_q(c->p.lattice) * c->hdom.ld * elem_size(c->p.storage);
  return bytes < 0xffffffffull;
}

int launch_one_step(rmrt_ctx* c, long long step_index, hipStream_t s) {
  StepLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.doms = c->ddoms + c->dom;
  a.tiles = nullptr;
  a.tile_nodes = (c->flags & STEP_WIDE_TILES) ? 512 : 256;
  a.ntiles = (c->hdom.N + a.tile_nodes - 1) / a.tile_nodes;
  a.flags = c->flags;
  if (!buffer_offsets_apply(c)) a.flags &= ~STEP_BUFFER_OFFSETS;
  a.parity = (uint32_t)(step_index & 1);
  a.eq = step_eq(c);
  a.force = step_force(c);
  a.bc = c->step_bc;
  a.phase = c->p.pattern == RMRT_AB ? PH_AB : ((step_index & 1) ? PH_AA_ODD : PH_AA_EVEN);
  a.grid = persistent_grid(a.ntiles, c->cus, c->blocks_per_cu, c->flags);
  a.lds_bytes = residency_lds(c->blocks_per_cu, c->flags);
  a.block = 256;
  a.stream = s;
  hipError_t e = dispatch_step(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "step launch failed: %s", hipGetErrorString(e));
  return RMRT_OK;
}

constexpr int kGraphChunk = 256;

// The graph of n launches starting at step `first`, cached by (n, parity of
// the first step): captured and instantiated on first use, and uploaded to
// stream s when one is given (rmrt_step_prepare).
int graph_for(rmrt_ctx* c, int n, long long first, hipGraphExec_t* out, hipStream_t upload) {
  const auto key = std::make_pair(n, (int)(first & 1));
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int rc = RMRT_OK;
    for (int i = 0; i < n && rc == RMRT_OK; ++i) rc = launch_one_step(c, first + i, c->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (rc != RMRT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(RMRT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(RMRT_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    if (c->graphs.size() >= 16) drop_graphs(c->graphs);
    it = c->graphs.emplace(key, ge).first;
    if (upload) HIP_TRY(hipGraphUpload(ge, upload));
  }
  *out = it->second;
  return RMRT_OK;
}

// steps n launches as a cached graph keyed by (n, parity of the first step)
int run_graph(rmrt_ctx* c, int n, hipStream_t s) {
  hipGraphExec_t ge = nullptr;
  int rc = graph_for(c, n, c->steps, &ge, nullptr);
  if (rc != RMRT_OK) return rc;
  HIP_TRY(hipGraphLaunch(ge, s));
  c->steps += n;
  return RMRT_OK;
}

// The graphs rmrt_step(n) would replay from step `first` (chunks of
// kGraphChunk, then the rest; a single step runs without a graph); returns
// the step count after them.
int prepare_graphs(rmrt_ctx* c, int n, long long first, hipStream_t s, long long* after) {
  hipGraphExec_t ge = nullptr;
  int left = n;
  while (left >= kGraphChunk) {
    int rc = graph_for(c, kGraphChunk, first, &ge, s);
    if (rc != RMRT_OK) return rc;
    first += kGraphChunk;
    left -= kGraphChunk;
  }
  if (left > 1) {
    int rc = graph_for(c, left, first, &ge, s);
    if (rc != RMRT_OK) return rc;
  }
  *after = first + left;
  return RMRT_OK;
}

int step_impl(rmrt_ctx* c, int nsteps, hipStream_t s) {
  if (nsteps == 1) {
    int rc = launch_one_step(c, c->steps, s);
    if (rc == RMRT_OK) c->steps += 1;
    return rc;
  }
  int left = nsteps;
  while (left >= kGraphChunk) {
    int rc = run_graph(c, kGraphChunk, s);
    if (rc != RMRT_OK) return rc;
    left -= kGraphChunk;
  }
  if (left > 1) return run_graph(c, left, s);
  if (left == 1) {
    int rc = launch_one_step(c, c->steps, s);
    if (rc == RMRT_OK) c->steps += 1;
    return rc;
  }
  return RMRT_OK;
}

int reduce_impl(rmrt_ctx* c, double out[4], hipStream_t s) {
  AuxLaunch a = aux_of(c, s);
  a.out0 = c->partials;
  hipError_t e = dispatch_reduce(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "reduce launch: %s", hipGetErrorString(e));
  e = launch_reduce_final(c->partials, a.grid, c->dres, 5, s);
  if (e != hipSuccess) return fail(RMRT_EHIP, "reduce final: %s", hipGetErrorString(e));
  HIP_TRY(hipMemcpyAsync(c->hres, c->dres, sizeof(double) * 5, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out[0] = c->hres[4] * c->p.rho0 + c->hres[0];
  out[1] = c->hres[1];
  out[2] = c->hres[2];
  out[3] = c->hres[3];
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(out[k])) return fail(RMRT_ENONFINITE, "non-finite reduction result");
  return RMRT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* rmrt_last_error(void) { return g_last_error.c_str(); }

const char* rmrt_version(void) { return "rmrt 0.1 (gfx950)"; }

int rmrt_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src) return fail(RMRT_EINVAL, "NULL pointer");
  if (bytes % 16) return fail(RMRT_EINVAL, "bytes must be a multiple of 16");
  hipError_t e = launch_stream_copy(dst, src, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RMRT_EHIP, "copy launch: %s", hipGetErrorString(e));
  return RMRT_OK;
}

int rmrt_derive(const rmrt_params* p, rmrt_derived* out) {
  Derived v;
  int rc = derive(p, v);
  if (rc != RMRT_OK) return rc;
  if (!out) return fail(RMRT_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->q = v.q;
  out->d = v.d;
  for (int a = 0; a < 3; ++a) out->c[a] = v.c[a];
  out->cs2 = v.cs2;
  for (int j = 0; j < 27; ++j) out->w[j] = v.w[j];
  out->s_nu = v.s_nu;
  for (int a = 0; a < 3; ++a) {
    out->s_s[a] = v.s_s[a];
    out->s_b[a] = v.s_b[a];
    for (int b = 0; b < 3; ++b) out->Sbar2[a][b] = v.Sbar[a][b];
  }
  out->s_hi = v.s_hi;
  out->nu_b = v.nu_b;
  for (int k = 0; k < 3; ++k) out->s_pair[k] = v.s_pair[k];
  return RMRT_OK;
}

int rmrt_population_bytes(const rmrt_params* p, size_t* bytes) {
  Derived v;
  int rc = derive(p, v);
  if (rc != RMRT_OK) return rc;
  if (!bytes) return fail(RMRT_EINVAL, "bytes is NULL");
  const uint32_t N = (uint32_t)p->n[0] * (uint32_t)p->n[1] * (uint32_t)p->n[2];
  *bytes = (size_t)v.q * stream_ld(N, p->storage) * elem_size(p->storage);
  return RMRT_OK;
}

static int ctx_create(rmrt_ctx** out, const rmrt_params* p, void* f0, void* f1, const uint8_t* solid,
                      DomainDev* ddoms, uint32_t dom) {
  if (!out) return fail(RMRT_EINVAL, "out is NULL");
  *out = nullptr;
  Derived v;
  int rc = derive(p, v);
  if (rc != RMRT_OK) return rc;
  if (!f0) return fail(RMRT_EINVAL, "f0 is NULL");
  if (p->pattern == RMRT_AB && !f1) return fail(RMRT_EINVAL, "RMRT_AB needs f1");
  if (p->pattern == RMRT_AA && f1) return fail(RMRT_EINVAL, "RMRT_AA takes f1 = NULL");
  rmrt_ctx* c = new (std::nothrow) rmrt_ctx();
  if (!c) return fail(RMRT_ENOMEM, "out of host memory");
  c->p = *p;
  c->v = v;
  fill_domain(p, v, c->hdom, f0, f1, solid);
  if (ddoms) {
    c->ddoms = ddoms;
    c->dom = dom;
    c->owns_ddoms = false;
  } else {
    hipError_t e = hipMalloc(&c->ddoms, sizeof(DomainDev));
    if (e != hipSuccess) {
      delete c;
      return fail(RMRT_EHIP, "hipMalloc(param block): %s", hipGetErrorString(e));
    }
    c->owns_ddoms = true;
    c->dom = 0;
  }
  rc = ctx_alloc_scratch(c);
  if (rc != RMRT_OK) {
    ctx_release(c);
    delete c;
    return rc;
  }
  if (c_zero_form(p)) {
    hipError_t e = hipMalloc(&c->hist, (p->storage == RMRT_F64 ? 8 : 4) * (size_t)c->hdom.N);
    if (e != hipSuccess) {
      ctx_release(c);
      delete c;
      return fail(RMRT_EHIP, "hipMalloc(history field): %s", hipGetErrorString(e));
    }
    c->hdom.hist = c->hist;
  }
  if (RMRT_CHECKED != 0) {
    hipError_t e = hipMalloc(&c->oob, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(c->oob, 0, sizeof(uint32_t));
    if (e != hipSuccess) {
      ctx_release(c);
      delete c;
      return fail(RMRT_EHIP, "hipMalloc(index-check counter): %s", hipGetErrorString(e));
    }
    c->hdom.oob = c->oob;
  }
  c->cus = device_cus();
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  {
    // set-up of the allocation-free reduction's scratch on this device; a
    // failure here is reported by rmrt_reduce_noalloc, the only user
    double* unused = nullptr;
    if (noalloc_scratch(c->device, &unused) != RMRT_OK) g_last_error.clear();
  }
  default_launch(*p, c->hdom.walls != 0 || c->hdom.has_solid, c->blocks_per_cu, c->flags);
  c->step_bc = c->hdom.walls != 0 ? 1 : 0;
  if (c->hdom.has_solid) {
    rc = alloc_links(c);
    if (rc != RMRT_OK) {
      ctx_release(c);
      delete c;
      return rc;
    }
  }
  *out = c;
  return RMRT_OK;
}

int rmrt_init(rmrt_ctx** out, const rmrt_params* p, void* f0, void* f1, const uint8_t* solid,
              const double* rho, const double* u, int with_fne, void* stream) {
  rmrt_ctx* c = nullptr;
  int rc = ctx_create(&c, p, f0, f1, solid, nullptr, 0);
  if (rc != RMRT_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(c->ddoms, &c->hdom, sizeof(DomainDev), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    ctx_release(c);
    delete c;
    return fail(RMRT_EHIP, "param upload: %s", hipGetErrorString(e));
  }
  if (!rho) {
    ctx_release(c);
    delete c;
    return fail(RMRT_EINVAL, "rho is NULL");
  }
  if (c->links) rc = build_links(c, s);
  if (rc == RMRT_OK) rc = launch_init_fields(c, rho, u, with_fne, s);
  if (rc != RMRT_OK) {
    ctx_release(c);
    delete c;
    return rc;
  }
  *out = c;
  return RMRT_OK;
}

int rmrt_set_fields(rmrt_ctx* c, const double* rho, const double* u, int with_fne, void* stream) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (!rho) return fail(RMRT_EINVAL, "rho is NULL");
  if (!c->batch) c->steps = 0;  // a standalone context restarts at an even step
  return launch_init_fields(c, rho, u, with_fne, (hipStream_t)stream);
}

int rmrt_set_source_fields(rmrt_ctx* c, const void* S, const void* F, void* stream) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (c->batch) return fail(RMRT_EINVAL, "source fields are not offered on the domains of a batch");
  if (F && c->p.equation != RMRT_NSE) return fail(RMRT_EINVAL, "a body-force field is an NSE input");
  hipStream_t s = (hipStream_t)stream;
  const size_t es = c->p.storage == RMRT_F64 ? 8 : 4;
  const size_t N = c->hdom.N;
  drop_graphs(c->graphs);   // cached graphs were captured for the previous source mode
  if (!S && !F) {
    c->hdom.src_field = 0;
    c->hdom.src = c->hdom.frc = nullptr;
    c->hdom.sprev = nullptr;
  } else {
    c->hdom.src_field = 1;
    c->hdom.src = S;
    c->hdom.frc = F;
    if (c->p.equation == RMRT_NCDE && c->p.gamma0) {
      // F(t - dt) of the gamma = 0 form: the attached source (no difference at the first step)
      if (!c->sprev) HIP_TRY(hipMalloc(&c->sprev, es * N));
      if (S)
        HIP_TRY(hipMemcpyAsync(c->sprev, S, es * N, hipMemcpyDeviceToDevice, s));
      else
        HIP_TRY(hipMemsetAsync(c->sprev, 0, es * N, s));
      c->hdom.sprev = c->sprev;
    } else {
      c->hdom.sprev = nullptr;
    }
  }
  HIP_TRY(hipMemcpyAsync(c->ddoms + c->dom, &c->hdom, sizeof(DomainDev), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RMRT_OK;
}

int rmrt_step(rmrt_ctx* c, int nsteps, void* stream) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (c->batch) return fail(RMRT_EINVAL, "domain belongs to a batch: use rmrt_batch_step");
  if (nsteps < 0) return fail(RMRT_EINVAL, "nsteps < 0");
  hipStream_t s = (hipStream_t)stream;
  if (c->p.check_every > 0) {
    int left = nsteps;
    while (left > 0) {
      const int k = std::min(left, c->p.check_every);
      int rc = step_impl(c, k, s);
      if (rc != RMRT_OK) return rc;
      left -= k;
      double r[4];
      rc = reduce_impl(c, r, s);
      if (rc != RMRT_OK) return rc;
    }
    return RMRT_OK;
  }
  return step_impl(c, nsteps, s);
}

int rmrt_step_prepare(rmrt_ctx* c, int nsteps, void* stream) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (c->batch) return fail(RMRT_EINVAL, "domain belongs to a batch: use rmrt_batch_step_prepare");
  if (nsteps < 0) return fail(RMRT_EINVAL, "nsteps < 0");
  hipStream_t s = (hipStream_t)stream;
  long long at = c->steps;
  if (c->p.check_every > 0) {
    int left = nsteps;
    while (left > 0) {
      const int k = std::min(left, c->p.check_every);
      int rc = prepare_graphs(c, k, at, s, &at);
      if (rc != RMRT_OK) return rc;
      left -= k;
    }
    return RMRT_OK;
  }
  return prepare_graphs(c, nsteps, at, s, &at);
}

int rmrt_moments(rmrt_ctx* c, void* rho_out, void* u_out, int out_dtype, void* stream) {
  if (!c || !rho_out) return fail(RMRT_EINVAL, "ctx or rho_out is NULL");
  if (out_dtype != RMRT_OUT_F64 && out_dtype != RMRT_OUT_F32) return fail(RMRT_EINVAL, "bad out_dtype");
  AuxLaunch a = aux_of(c, (hipStream_t)stream);
  a.out0 = rho_out;
  a.out1 = u_out;
  a.flag = out_dtype == RMRT_OUT_F32;
  hipError_t e = dispatch_moments(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "moments launch: %s", hipGetErrorString(e));
  return RMRT_OK;
}

}  // extern "C"

namespace {
int check_local_args(const rmrt_ctx* c, int kind, const void* out, int out_dtype) {
  if (!c || !out) return fail(RMRT_EINVAL, "ctx or out is NULL");
  if (c->hdom.src_field)
    return fail(RMRT_EUNSUPPORTED, "local outputs take the parameter set's constant sources (fields attached)");
  if (c->p.central || c->p.hermite || c->p.bhll)
    return fail(RMRT_EUNSUPPORTED, "local outputs are built for the raw-moment collision");
  if (out_dtype != RMRT_OUT_F64 && out_dtype != RMRT_OUT_F32) return fail(RMRT_EINVAL, "bad out_dtype");
  const bool nse = c->p.equation == RMRT_NSE;
  if (kind == RMRT_GRAD_STRAIN || kind == RMRT_GRAD_STRESS) {
    if (!nse) return fail(RMRT_EINVAL, "strain rate and stress are NSE outputs");
  } else if (kind == RMRT_GRAD_PHI) {
    if (nse) return fail(RMRT_EINVAL, "grad phi is an NCDE output");
  } else {
    return fail(RMRT_EINVAL, "unknown kind %d", kind);
  }
  return RMRT_OK;
}
}  // namespace

extern "C" {

int rmrt_local_gradients(rmrt_ctx* c, int kind, void* out, int out_dtype, void* stream) {
  int rc = check_local_args(c, kind, out, out_dtype);
  if (rc != RMRT_OK) return rc;
  AuxLaunch a = aux_of(c, (hipStream_t)stream);
  a.out0 = out;
  a.flag = out_dtype == RMRT_OUT_F32;
  a.kind = kind;
  // one node per thread (measured at 256 x 256 x 128: 147-153 us against
  // 162-170 us for a 2048-block grid-stride loop)
  a.grid = (c->hdom.N + kAuxBlock - 1) / kAuxBlock;
  hipError_t e = dispatch_local(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "local gradients launch: %s", hipGetErrorString(e));
  return RMRT_OK;
}

int rmrt_step_local(rmrt_ctx* c, int kind, void* out, int out_dtype, void* stream) {
  int rc = check_local_args(c, kind, out, out_dtype);
  if (rc != RMRT_OK) return rc;
  if (c->batch) return fail(RMRT_EINVAL, "domain belongs to a batch");
  hipStream_t s = (hipStream_t)stream;
  StepLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.doms = c->ddoms + c->dom;
  a.tiles = nullptr;
  a.tile_nodes = 256;
  a.ntiles = (c->hdom.N + a.tile_nodes - 1) / a.tile_nodes;
  a.flags = c->flags & STEP_ALTERNATE_ORDER;
  a.parity = (uint32_t)(c->steps & 1);
  a.eq = step_eq(c);
  a.force = step_force(c);
  a.bc = c->step_bc;
  a.phase = c->p.pattern == RMRT_AB ? PH_AB : ((c->steps & 1) ? PH_AA_ODD : PH_AA_EVEN);
  a.grid = a.ntiles;
  a.lds_bytes = (c->flags & STEP_PERSISTENT) ? 0u : residency_lds(c->blocks_per_cu, 0u);
  a.block = 256;
  a.stream = s;
  a.local_out = out;
  a.local_kind = kind;
  a.local_f32 = out_dtype == RMRT_OUT_F32;
  hipError_t e = dispatch_step(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "fused step launch failed: %s", hipGetErrorString(e));
  c->steps += 1;
  return RMRT_OK;
}

int rmrt_populations(rmrt_ctx* c, double* f_out, void* stream) {
  if (!c || !f_out) return fail(RMRT_EINVAL, "ctx or f_out is NULL");
  AuxLaunch a = aux_of(c, (hipStream_t)stream);
  a.out0 = f_out;
  hipError_t e = dispatch_populations(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "populations launch: %s", hipGetErrorString(e));
  return RMRT_OK;
}

int rmrt_reduce(rmrt_ctx* c, double out[4], void* stream) {
  if (!c || !out) return fail(RMRT_EINVAL, "ctx or out is NULL");
  return reduce_impl(c, out, (hipStream_t)stream);
}

int rmrt_reduce_noalloc(rmrt_ctx* c, double* out, void* stream) {
  if (!c || !out) return fail(RMRT_EINVAL, "ctx or out is NULL");
  double* part = nullptr;
  int rc = noalloc_scratch(c->device, &part);
  if (rc != RMRT_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  AuxLaunch a = aux_of(c, s);
  if (a.grid > kNoAllocBlocks)
    return fail(RMRT_EINVAL, "the reduction needs %u partial blocks; the allocation-free scratch holds %u",
                a.grid, kNoAllocBlocks);
  a.out0 = part;
  hipError_t e = dispatch_reduce(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "reduce launch: %s", hipGetErrorString(e));
  e = launch_reduce_final_mass(part, a.grid, c->p.rho0, out, s);
  if (e != hipSuccess) return fail(RMRT_EHIP, "reduce final: %s", hipGetErrorString(e));
  return RMRT_OK;
}

int rmrt_residual(rmrt_ctx* c, double* r, void* stream) {
  if (!c || !r) return fail(RMRT_EINVAL, "ctx or r is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int K = c->p.equation == RMRT_NSE ? c->v.d : 1;
  if (!c->uprev) HIP_TRY(hipMalloc(&c->uprev, sizeof(double) * (size_t)K * c->hdom.N));
  AuxLaunch a = aux_of(c, s);
  a.out0 = c->partials;
  a.out1 = c->uprev;
  a.flag = c->have_prev ? 1 : 0;
  hipError_t e = dispatch_residual(c->p.lattice, c->p.storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "residual launch: %s", hipGetErrorString(e));
  e = launch_reduce_final(c->partials, a.grid, c->dres, 2, s);
  if (e != hipSuccess) return fail(RMRT_EHIP, "residual final: %s", hipGetErrorString(e));
  HIP_TRY(hipMemcpyAsync(c->hres, c->dres, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const bool first = !c->have_prev;
  c->have_prev = true;
  if (!std::isfinite(c->hres[0]) || !std::isfinite(c->hres[1]))
    return fail(RMRT_ENONFINITE, "non-finite residual");
  if (first) {
    *r = INFINITY;
  } else {
    *r = c->hres[1] > 0 ? std::sqrt(c->hres[0] / c->hres[1]) : (c->hres[0] > 0 ? INFINITY : 0.0);
  }
  return RMRT_OK;
}

int rmrt_steps_taken(const rmrt_ctx* c, long long* steps) {
  if (!c || !steps) return fail(RMRT_EINVAL, "NULL argument");
  *steps = c->steps;
  return RMRT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Checkpoints: a header, then the stored populations of the current state in
// their stored layout (one buffer: the AA buffer, or the AB buffer the step
// count selects), then the C = 0 history field and the gamma = 0
// previous-step source when the context has them.
// ---------------------------------------------------------------------------
namespace {
constexpr uint64_t kCkptMagic = 0x3150434b54524d52ull;   // "RMRTCKP1"
struct CkptHeader {
  uint64_t magic;
  int32_t lattice, equation, storage, pattern, n[3], c_zero;
  uint32_t ld, has_hist, has_sprev, pad;
  int64_t steps;
  uint64_t pop_bytes, field_bytes;
};
static_assert(sizeof(CkptHeader) % 16 == 0, "checkpoint payload stays 16-byte aligned");

CkptHeader ckpt_header(const rmrt_ctx* c) {
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kCkptMagic;
  h.lattice = c->p.lattice;
  h.equation = c->p.equation;
  h.storage = c->p.storage;
  h.pattern = c->p.pattern;
  for (int a = 0; a < 3; ++a) h.n[a] = c->p.n[a];
  h.c_zero = c->p.c_zero ? 1 : 0;
  h.ld = c->hdom.ld;
  h.has_hist = c->hist != nullptr;
  h.has_sprev = c->hdom.sprev != nullptr;
  h.steps = c->steps;
  h.pop_bytes = (uint64_t)lattice_q(c->p.lattice) * c->hdom.ld * elem_size(c->p.storage);
  h.field_bytes = (uint64_t)c->hdom.N * (c->p.storage == RMRT_F64 ? 8 : 4);
  return h;
}
size_t ckpt_bytes(const CkptHeader& h) {
  return sizeof(CkptHeader) + h.pop_bytes + (h.has_hist + h.has_sprev) * h.field_bytes;
}
void* current_population_buffer(const rmrt_ctx* c) {
  return (c->p.pattern == RMRT_AB && (c->steps & 1)) ? c->hdom.fb : c->hdom.fa;
}
}  // namespace

extern "C" {

int rmrt_checkpoint_bytes(const rmrt_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(RMRT_EINVAL, "NULL argument");
  *bytes = ckpt_bytes(ckpt_header(c));
  return RMRT_OK;
}

int rmrt_checkpoint_save(rmrt_ctx* c, void* dst, void* stream) {
  if (!c || !dst) return fail(RMRT_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const CkptHeader h = ckpt_header(c);
  char* out = (char*)dst;
  HIP_TRY(hipMemcpyAsync(out, &h, sizeof(h), hipMemcpyDefault, s));
  size_t off = sizeof(h);
  HIP_TRY(hipMemcpyAsync(out + off, current_population_buffer(c), h.pop_bytes, hipMemcpyDefault, s));
  off += h.pop_bytes;
  if (h.has_hist) {
    HIP_TRY(hipMemcpyAsync(out + off, c->hist, h.field_bytes, hipMemcpyDefault, s));
    off += h.field_bytes;
  }
  if (h.has_sprev) HIP_TRY(hipMemcpyAsync(out + off, c->hdom.sprev, h.field_bytes, hipMemcpyDefault, s));
  HIP_TRY(hipStreamSynchronize(s));   // the header copy reads a host local
  return RMRT_OK;
}

int rmrt_checkpoint_restore(rmrt_ctx* c, const void* src, void* stream) {
  if (!c || !src) return fail(RMRT_EINVAL, "NULL argument");
  if (c->batch) return fail(RMRT_EINVAL, "domain belongs to a batch: its step count is the batch's");
  hipStream_t s = (hipStream_t)stream;
  CkptHeader h;
  HIP_TRY(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDefault, s));
  HIP_TRY(hipStreamSynchronize(s));
  const CkptHeader mine = ckpt_header(c);
  if (h.magic != kCkptMagic) return fail(RMRT_EINVAL, "not a checkpoint of this library");
  if (h.lattice != mine.lattice || h.equation != mine.equation || h.storage != mine.storage ||
      h.pattern != mine.pattern || h.n[0] != mine.n[0] || h.n[1] != mine.n[1] || h.n[2] != mine.n[2] ||
      h.c_zero != mine.c_zero || h.ld != mine.ld)
    return fail(RMRT_EINVAL, "checkpoint of a different lattice, equation, storage, pattern or size");
  if (h.has_hist != mine.has_hist || h.has_sprev != mine.has_sprev)
    return fail(RMRT_EINVAL, "checkpoint %s a previous-step source field the context %s",
                h.has_sprev ? "holds" : "lacks", mine.has_sprev ? "has" : "has not");
  if (h.steps < 0) return fail(RMRT_EINVAL, "checkpoint step count %lld < 0", (long long)h.steps);
  const char* in = (const char*)src;
  size_t off = sizeof(h);
  c->steps = h.steps;   // selects the layout (AA) or the buffer (AB) written next
  HIP_TRY(hipMemcpyAsync(current_population_buffer(c), in + off, h.pop_bytes, hipMemcpyDefault, s));
  off += h.pop_bytes;
  if (h.has_hist) {
    HIP_TRY(hipMemcpyAsync(c->hist, in + off, h.field_bytes, hipMemcpyDefault, s));
    off += h.field_bytes;
  }
  if (h.has_sprev) HIP_TRY(hipMemcpyAsync(c->hdom.sprev, in + off, h.field_bytes, hipMemcpyDefault, s));
  c->have_prev = false;   // the residual restarts from the restored state
  HIP_TRY(hipStreamSynchronize(s));
  return RMRT_OK;
}

int rmrt_set_launch(rmrt_ctx* c, int blocks_per_cu, int flags) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (blocks_per_cu < 0 || blocks_per_cu > 32) return fail(RMRT_EINVAL, "blocks_per_cu must be in [0, 32]");
  if (flags & ~63) return fail(RMRT_EINVAL, "unknown launch flags 0x%x", flags);
  if (blocks_per_cu == 1 && !(flags & STEP_PERSISTENT))
    return fail(RMRT_EINVAL, "a residency cap of 1 workgroup per CU is not supported (use >= 2)");
  c->blocks_per_cu = blocks_per_cu;
  c->flags = (uint32_t)flags;
  drop_graphs(c->graphs);
  return RMRT_OK;
}

int rmrt_get_launch(const rmrt_ctx* c, int* blocks_per_cu, int* flags) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (blocks_per_cu) *blocks_per_cu = c->blocks_per_cu;
  if (flags) *flags = (int)c->flags;
  return RMRT_OK;
}

int rmrt_tune(rmrt_ctx* c, int steps, void* stream, int* blocks_per_cu) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (c->batch) return fail(RMRT_EINVAL, "domain belongs to a batch: use rmrt_batch_autotune");
  if (steps < 1) return fail(RMRT_EINVAL, "steps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int cands[] = {0, 2, 3, 4, 5, 6, 8};
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.e0));
  HIP_TRY(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  int best = kDefaultBlocksPerCU, best_flags = 0;
  float best_ms = 1e30f;
  const int nbuf = buffer_offsets_apply(c) ? 2 : 1;
  const int nchunk = rows_straddle_lines(c->p) ? 2 : 1;
  for (int chunk = 0; chunk < nchunk; ++chunk)
  for (int buf = 0; buf < nbuf; ++buf)
  for (int wide = 0; wide < 2; ++wide)
  for (int k : cands) {
    const int fl = (wide ? (int)STEP_WIDE_TILES : 0) | (buf ? (int)STEP_BUFFER_OFFSETS : 0) |
                   (chunk ? (int)STEP_XCD_CHUNKS : 0) | (int)STEP_ALTERNATE_ORDER;
    int rc = rmrt_set_launch(c, k, fl);
    if (rc == RMRT_OK) rc = step_impl(c, 2, s);
    if (rc == RMRT_OK) rc = step_impl(c, steps, s);
    if (rc != RMRT_OK) return rc;
    HIP_TRY(hipEventRecord(e0, s));
    rc = step_impl(c, steps, s);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    if (rc != RMRT_OK) return rc;
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = k;
      best_flags = fl;
    }
  }
  if (blocks_per_cu) *blocks_per_cu = best;
  return rmrt_set_launch(c, best, best_flags);
}

int rmrt_free(rmrt_ctx* c) {
  if (!c) return RMRT_OK;
  if (c->batch) return fail(RMRT_EINVAL, "domain belongs to a batch: use rmrt_batch_free");
  ctx_release(c);
  delete c;
  return RMRT_OK;
}

}  // extern "C"

namespace {
struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};
struct CtxGuard {
  rmrt_ctx* c = nullptr;
  ~CtxGuard() {
    if (c) (void)rmrt_free(c);
  }
};
// uniform in [-1, 1) from a counter (splitmix64 finaliser)
double noise(uint64_t k) {
  uint64_t z = k + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
}  // namespace

extern "C" {

// Linear (von Neumann) stability preflight: the parameter set's own step
// kernel, in FP64 on a periodic 16^d domain without walls, solids or
// forcing, evolves a small zero-mean perturbation of the uniform state
// (rho0, u0), renormalised to its initial size after every leg of an even
// number of steps (a power iteration of the linearised collide-and-stream
// operator; even legs end in the natural AA layout, so the stored values are
// read and rescaled in place).  The mean growth per step over the second
// half of the legs estimates the largest amplification factor |lambda(k)|
// over the domain's wave vectors.
int rmrt_preflight(const rmrt_params* p, const double* u0, int steps, double* growth, void* stream) {
  if (!p || !growth) return fail(RMRT_EINVAL, "params or growth is NULL");
  if (steps < 16 || steps > 1000000) return fail(RMRT_EINVAL, "steps must be in [16, 1000000]");
  hipStream_t s = (hipStream_t)stream;
  rmrt_params q = *p;
  q.storage = RMRT_F64;
  q.pattern = RMRT_AA;
  q.wall_faces = 0;
  q.check_every = 0;
  q.source = 0.0;
  for (int a = 0; a < 3; ++a) q.force[a] = 0.0;
  q.n[0] = q.n[1] = 16;
  q.n[2] = lattice_2d(q.lattice) ? 1 : 16;
  Derived v;
  int rc = derive(&q, v);
  if (rc != RMRT_OK) return rc;
  const size_t N = (size_t)q.n[0] * q.n[1] * q.n[2];
  const int Q = v.q;
  size_t bytes = 0;
  rc = rmrt_population_bytes(&q, &bytes);
  if (rc != RMRT_OK) return rc;
  const size_t ld = bytes / (sizeof(double) * (size_t)Q);
  DevMem f, rho_d, u_d;
  HIP_TRY(hipMalloc(&f.p, bytes));
  HIP_TRY(hipMalloc(&rho_d.p, N * sizeof(double)));
  HIP_TRY(hipMalloc(&u_d.p, 3 * N * sizeof(double)));
  std::vector<double> h_rho(N, q.rho0), h_u(3 * N, 0.0);
  if (u0 && q.equation == RMRT_NSE)
    for (int a = 0; a < v.d; ++a) std::fill(h_u.begin() + a * N, h_u.begin() + (a + 1) * N, u0[a]);
  HIP_TRY(hipMemcpyAsync(rho_d.p, h_rho.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(u_d.p, h_u.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
  CtxGuard g;
  rc = rmrt_init(&g.c, &q, f.p, nullptr, nullptr, (const double*)rho_d.p, (const double*)u_d.p, 0, stream);
  if (rc != RMRT_OK) return rc;
  // state = stored populations [+ the C = 0 form's previous-step phi]
  double* hist = (double*)g.c->hdom.hist;
  const size_t nh = hist ? N : 0;
  std::vector<double> base((size_t)Q * ld + nh), cur(base.size());
  HIP_TRY(hipMemcpyAsync(base.data(), f.p, bytes, hipMemcpyDeviceToHost, s));
  if (hist) HIP_TRY(hipMemcpyAsync(base.data() + (size_t)Q * ld, hist, nh * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // the uniform state is a fixed point of the step; perturb every stored
  // population by a zero-mean pseudo-random field of amplitude 1e-7
  cur = base;
  for (int j = 0; j < Q; ++j) {
    double mean = 0;
    for (size_t n = 0; n < N; ++n) mean += noise((uint64_t)j * N + n);
    mean /= (double)N;
    for (size_t n = 0; n < N; ++n) cur[(size_t)j * ld + n] += 1e-7 * (noise((uint64_t)j * N + n) - mean);
  }
  auto dev_norm = [&]() {
    double acc = 0;
    for (int j = 0; j < Q; ++j)
      for (size_t n = 0; n < N; ++n) {
        const double d = cur[(size_t)j * ld + n] - base[(size_t)j * ld + n];
        acc += d * d;
      }
    for (size_t n = 0; n < nh; ++n) {
      const double d = cur[(size_t)Q * ld + n] - base[(size_t)Q * ld + n];
      acc += d * d;
    }
    return std::sqrt(acc);
  };
  const double norm0 = dev_norm();
  const int legs = 8;
  const int L = std::max(2, (steps / legs + 1) / 2 * 2);
  double log_growth = 0;
  for (int leg = 0; leg < legs; ++leg) {
    HIP_TRY(hipMemcpyAsync(f.p, cur.data(), bytes, hipMemcpyHostToDevice, s));
    if (hist) HIP_TRY(hipMemcpyAsync(hist, cur.data() + (size_t)Q * ld, nh * sizeof(double), hipMemcpyHostToDevice, s));
    rc = rmrt_step(g.c, L, stream);
    if (rc != RMRT_OK) return rc;
    HIP_TRY(hipMemcpyAsync(cur.data(), f.p, bytes, hipMemcpyDeviceToHost, s));
    if (hist) HIP_TRY(hipMemcpyAsync(cur.data() + (size_t)Q * ld, hist, nh * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double nrm = dev_norm();
    if (!std::isfinite(nrm)) {
      *growth = INFINITY;
      return RMRT_OK;
    }
    if (nrm == 0.0) {
      *growth = 0.0;
      return RMRT_OK;
    }
    if (leg >= legs / 2) log_growth += std::log(nrm / norm0);
    const double scale = norm0 / nrm;
    for (size_t i = 0; i < cur.size(); ++i) cur[i] = base[i] + (cur[i] - base[i]) * scale;
  }
  *growth = std::exp(log_growth / ((double)L * (legs - legs / 2)));
  return RMRT_OK;
}

int rmrt_checked_build(void) { return RMRT_CHECKED != 0 ? 1 : 0; }

int rmrt_checked_violations(rmrt_ctx* c, unsigned* count, void* stream) {
  if (!c || !count) return fail(RMRT_EINVAL, "ctx or count is NULL");
  if (RMRT_CHECKED == 0 || !c->oob) return fail(RMRT_EUNSUPPORTED, "not a checked build");
  hipStream_t s = (hipStream_t)stream;
  uint32_t v = 0;
  HIP_TRY(hipMemcpyAsync(&v, c->oob, sizeof(v), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *count = v;
  return RMRT_OK;
}

int rmrt_checked_set_limit(rmrt_ctx* c, unsigned limit, void* stream) {
  if (!c) return fail(RMRT_EINVAL, "ctx is NULL");
  if (RMRT_CHECKED == 0 || !c->oob) return fail(RMRT_EUNSUPPORTED, "not a checked build");
  if (limit < 1 || limit > c->hdom.N) return fail(RMRT_EINVAL, "limit must be in [1, N]");
  hipStream_t s = (hipStream_t)stream;
  c->hdom.oob_limit = limit;
  HIP_TRY(hipMemsetAsync(c->oob, 0, sizeof(uint32_t), s));
  HIP_TRY(hipMemcpyAsync(c->ddoms + c->dom, &c->hdom, sizeof(DomainDev), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RMRT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched persistent stepping
// ---------------------------------------------------------------------------
namespace {

struct TileConfig {
  int threads, tile_nodes, blocks_per_cu;  // blocks_per_cu <= 0: one workgroup per tile
  int persistent;  // 1: persistent grid of blocks_per_cu per CU; 0: one workgroup per tile,
                   //    blocks_per_cu > 0 caps residency through dynamic LDS
  int nodes_per_thread;  // 1, or 2: two nodes read before either collides
};
// threads per block never exceed the kernels' launch bound of 256
constexpr int kMaxThreads = 256;
const TileConfig kTileShapes[] = {
    {256, 256, 0, 0, 1},  {256, 256, 2, 0, 1},  {256, 256, 3, 0, 1},  {256, 256, 4, 0, 1},
    {256, 256, 2, 1, 1},  {256, 256, 3, 1, 1},  {256, 1024, 2, 1, 1}, {256, 1024, 4, 1, 1},
    {256, 2048, 8, 1, 1}, {128, 512, 4, 1, 1},  {256, 512, 0, 0, 2},  {256, 512, 2, 0, 2},
    {256, 512, 3, 0, 2},  {256, 512, 4, 0, 2},  {256, 1024, 2, 1, 2}, {256, 1024, 3, 1, 2},
};
constexpr int kNumTileShapes = sizeof(kTileShapes) / sizeof(kTileShapes[0]);

}  // namespace

struct rmrt_batch {
  int nd = 0;
  std::vector<rmrt_ctx*> ctxs;
  DomainDev* ddoms = nullptr;
  Tile* dtiles = nullptr;
  uint32_t ntiles = 0;
  int cfg = 1;
  int cus = 256;
  long long steps = 0;
  int lattice = 0, storage = 0, equation = 0, pattern = 0, force = 0, bc = 0;
  std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
  hipStream_t cap = nullptr;
  // domain groups: consecutive domains whose population buffers add up to at
  // most group_bytes (0: one group) as (first tile, tile count); a stepping
  // call advances each group through all its steps before the next group
  size_t group_bytes = 0;
  std::vector<std::pair<uint32_t, uint32_t>> groups;
  // XCD chunks (STEP_XCD_CHUNKS) for the one-workgroup-per-tile launches of
  // the groups holding a domain whose rows straddle cache lines (mode 1, the
  // default), or never (mode 0)
  int xcd_chunks = 1;
  std::vector<uint8_t> group_chunked;
  double* dres_all = nullptr;  // 2 * nd residual sums (device)
  double* hres_all = nullptr;  // pinned host copy
};

namespace {

// Group consecutive domains (tiles are in domain order) up to group_bytes of
// population buffers each; a larger domain forms a group of its own.
void batch_make_groups(rmrt_batch* b) {
  b->groups.clear();
  b->group_chunked.clear();
  const uint32_t tn = (uint32_t)kTileShapes[b->cfg].tile_nodes;
  uint32_t first = 0, count = 0;
  size_t bytes = 0;
  bool straddle = false;
  for (int d = 0; d < b->nd; ++d) {
    const rmrt_ctx* c = b->ctxs[d];
    const uint32_t nt = (c->hdom.N + tn - 1) / tn;
    const size_t db = (size_t)lattice_q(c->p.lattice) * c->hdom.ld * elem_size(c->p.storage) *
                      (c->p.pattern == RMRT_AB ? 2u : 1u);
    if (b->group_bytes > 0 && count > 0 && bytes + db > b->group_bytes) {
      b->groups.emplace_back(first, count);
      b->group_chunked.push_back(straddle ? 1 : 0);
      first += count;
      count = 0;
      bytes = 0;
      straddle = false;
    }
    count += nt;
    bytes += db;
    straddle = straddle || rows_straddle_lines(c->p);
  }
  if (count > 0) {
    b->groups.emplace_back(first, count);
    b->group_chunked.push_back(straddle ? 1 : 0);
  }
  drop_graphs(b->graphs);
}

int batch_build_tiles(rmrt_batch* b, int cfg, hipStream_t s) {
  const TileConfig& tc = kTileShapes[cfg];
  std::vector<Tile> tiles;
  for (int d = 0; d < b->nd; ++d) {
    const uint32_t N = b->ctxs[d]->hdom.N;
    for (uint32_t st = 0; st < N; st += (uint32_t)tc.tile_nodes) {
      Tile t;
      t.dom = (uint32_t)d;
      t.start = st;
      t.count = std::min<uint32_t>((uint32_t)tc.tile_nodes, N - st);
      t.pad = 0;
      tiles.push_back(t);
    }
  }
  if (b->dtiles) {
    // a step launched earlier on any stream may still read the old tile list
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(b->dtiles));
    b->dtiles = nullptr;
  }
  HIP_TRY(hipMalloc(&b->dtiles, sizeof(Tile) * tiles.size()));
  HIP_TRY(hipMemcpyAsync(b->dtiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  b->ntiles = (uint32_t)tiles.size();
  b->cfg = cfg;
  batch_make_groups(b);
  return RMRT_OK;
}

int batch_launch(rmrt_batch* b, long long step_index, hipStream_t s, size_t group) {
  const TileConfig& tc = kTileShapes[b->cfg];
  StepLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.doms = b->ddoms;
  a.tiles = b->dtiles + b->groups[group].first;
  a.ntiles = b->groups[group].second;
  a.tile_nodes = (uint32_t)tc.tile_nodes;
  a.parity = (uint32_t)(step_index & 1);
  a.eq = b->equation;
  a.force = b->force;
  a.bc = b->bc;
  a.phase = b->pattern == RMRT_AB ? PH_AB : ((step_index & 1) ? PH_AA_ODD : PH_AA_EVEN);
  if (tc.threads > kMaxThreads) return fail(RMRT_EINVAL, "config uses %d threads > %d", tc.threads, kMaxThreads);
  a.flags = (tc.persistent && tc.blocks_per_cu > 0) ? (STEP_PERSISTENT | STEP_XCD_ORDER) : 0u;
  if (tc.nodes_per_thread == 2) a.flags |= STEP_WIDE_TILES;
  bool buf = true;
  for (const rmrt_ctx* c : b->ctxs) buf = buf && buffer_offsets_apply(c);
  if (buf) a.flags |= STEP_BUFFER_OFFSETS;
  a.flags |= STEP_ALTERNATE_ORDER;
  if (b->xcd_chunks && b->group_chunked[group] && !(a.flags & STEP_PERSISTENT)) a.flags |= STEP_XCD_CHUNKS;
  a.grid = persistent_grid(a.ntiles, b->cus, tc.blocks_per_cu, a.flags);
  a.lds_bytes = residency_lds(tc.blocks_per_cu, a.flags);
  a.block = (unsigned)tc.threads;
  a.stream = s;
  hipError_t e = dispatch_step(b->lattice, b->storage, a);
  if (e != hipSuccess) return fail(RMRT_EHIP, "batch step launch: %s", hipGetErrorString(e));
  return RMRT_OK;
}

void batch_advance(rmrt_batch* b, int n) {
  b->steps += n;
  for (auto* c : b->ctxs) c->steps = b->steps;
}

// The graph of n steps of every group from step `first`, cached by (n,
// parity, tile configuration); uploaded to stream `upload` when given.
int batch_graph_for(rmrt_batch* b, int n, long long first, hipGraphExec_t* out, hipStream_t upload) {
  const auto key = std::make_tuple(n, (int)(first & 1), b->cfg);
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = RMRT_OK;
    for (size_t gi = 0; gi < b->groups.size() && rc == RMRT_OK; ++gi)
      for (int i = 0; i < n && rc == RMRT_OK; ++i) rc = batch_launch(b, first + i, b->cap, gi);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != RMRT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(RMRT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(RMRT_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    if (b->graphs.size() >= 16) drop_graphs(b->graphs);
    it = b->graphs.emplace(key, ge).first;
    if (upload) HIP_TRY(hipGraphUpload(ge, upload));
  }
  *out = it->second;
  return RMRT_OK;
}

int batch_graph(rmrt_batch* b, int n, hipStream_t s) {
  hipGraphExec_t ge = nullptr;
  int rc = batch_graph_for(b, n, b->steps, &ge, nullptr);
  if (rc != RMRT_OK) return rc;
  HIP_TRY(hipGraphLaunch(ge, s));
  batch_advance(b, n);
  return RMRT_OK;
}

int batch_step_impl(rmrt_batch* b, int nsteps, hipStream_t s) {
  int left = nsteps;
  while (left >= kGraphChunk) {
    int rc = batch_graph(b, kGraphChunk, s);
    if (rc != RMRT_OK) return rc;
    left -= kGraphChunk;
  }
  if (left > 1) return batch_graph(b, left, s);
  if (left == 1) {
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      int rc = batch_launch(b, b->steps, s, gi);
      if (rc != RMRT_OK) return rc;
    }
    batch_advance(b, 1);
  }
  return RMRT_OK;
}

void batch_release(rmrt_batch* b) {
  (void)hipDeviceSynchronize();  // work issued on any stream may still use the buffers
  drop_graphs(b->graphs);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (auto* c : b->ctxs) {
    if (!c) continue;
    c->batch = nullptr;
    ctx_release(c);
    delete c;
  }
  b->ctxs.clear();
  if (b->dtiles) (void)hipFree(b->dtiles);
  if (b->ddoms) (void)hipFree(b->ddoms);
  if (b->dres_all) (void)hipFree(b->dres_all);
  if (b->hres_all) (void)hipHostFree(b->hres_all);
}

}  // namespace

extern "C" {

int rmrt_batch_num_configs(void) { return kNumTileShapes; }

int rmrt_batch_config_info(int cfg, int* threads, int* tile_nodes, int* blocks_per_cu, int* persistent,
                           int* nodes_per_thread) {
  if (cfg < 0 || cfg >= kNumTileShapes) return fail(RMRT_EINVAL, "config %d out of range", cfg);
  if (nodes_per_thread) *nodes_per_thread = kTileShapes[cfg].nodes_per_thread;
  if (threads) *threads = kTileShapes[cfg].threads;
  if (tile_nodes) *tile_nodes = kTileShapes[cfg].tile_nodes;
  if (blocks_per_cu) *blocks_per_cu = kTileShapes[cfg].blocks_per_cu;
  if (persistent) *persistent = kTileShapes[cfg].persistent;
  return RMRT_OK;
}

int rmrt_batch_create(rmrt_batch** out, int nd, const rmrt_params* params, void* const* f0, void* const* f1,
                      const uint8_t* const* solid, void* stream) {
  if (!out) return fail(RMRT_EINVAL, "out is NULL");
  *out = nullptr;
  if (nd < 1 || !params || !f0) return fail(RMRT_EINVAL, "need nd >= 1, params and f0");
  const rmrt_params& p0 = params[0];
  for (int d = 1; d < nd; ++d) {
    const rmrt_params& p = params[d];
    if (p.lattice != p0.lattice || p.equation != p0.equation || p.storage != p0.storage ||
        p.pattern != p0.pattern || (p.c_zero != 0) != (p0.c_zero != 0) || (p.central != 0) != (p0.central != 0) ||
        (p.hermite != 0) != (p0.hermite != 0) || (p.bhll != 0) != (p0.bhll != 0))
      return fail(RMRT_EINVAL, "domain %d differs in lattice/equation/storage/pattern/c_zero/central/hermite/bhll", d);
  }
  hipStream_t s = (hipStream_t)stream;
  rmrt_batch* b = new (std::nothrow) rmrt_batch();
  if (!b) return fail(RMRT_ENOMEM, "out of host memory");
  b->nd = nd;
  b->lattice = p0.lattice;
  b->storage = p0.storage;
  b->equation = p0.equation;
  b->pattern = p0.pattern;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->cus = prop.multiProcessorCount;
  hipError_t e = hipMalloc(&b->ddoms, sizeof(DomainDev) * nd);
  if (e != hipSuccess) {
    delete b;
    return fail(RMRT_EHIP, "hipMalloc(param blocks): %s", hipGetErrorString(e));
  }
  std::vector<DomainDev> host(nd);
  for (int d = 0; d < nd; ++d) {
    rmrt_ctx* c = nullptr;
    const uint8_t* sd = solid ? solid[d] : nullptr;
    int rc = ctx_create(&c, &params[d], f0[d], f1 ? f1[d] : nullptr, sd, b->ddoms, (uint32_t)d);
    if (rc != RMRT_OK) {
      batch_release(b);
      delete b;
      return rc;
    }
    c->batch = b;
    b->ctxs.push_back(c);
    b->equation = step_eq(c);
    b->force |= has_force(&params[d]) ? 1 : 0;
    b->bc = std::max(b->bc, c->step_bc);
  }
  // one boundary mode per batch: link bits everywhere when any domain has a solid mask
  for (int d = 0; d < nd; ++d) {
    rmrt_ctx* c = b->ctxs[d];
    if (b->bc == 2 && !c->links) {
      int rc2 = alloc_links(c);
      if (rc2 != RMRT_OK) {
        batch_release(b);
        delete b;
        return rc2;
      }
    }
    c->step_bc = b->bc;
    host[d] = c->hdom;
  }
  e = hipMemcpyAsync(b->ddoms, host.data(), sizeof(DomainDev) * nd, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    batch_release(b);
    delete b;
    return fail(RMRT_EHIP, "param upload: %s", hipGetErrorString(e));
  }
  int rc = batch_build_tiles(b, 1, s);
  for (int d = 0; d < nd && rc == RMRT_OK; ++d)
    if (b->ctxs[d]->links) rc = build_links(b->ctxs[d], s);
  for (int d = 0; d < nd && rc == RMRT_OK; ++d) rc = launch_init_fields(b->ctxs[d], nullptr, nullptr, 0, s);
  if (rc != RMRT_OK) {
    batch_release(b);
    delete b;
    return rc;
  }
  *out = b;
  return RMRT_OK;
}

int rmrt_batch_domain(rmrt_batch* b, int d, rmrt_ctx** out) {
  if (!b || !out || d < 0 || d >= b->nd) return fail(RMRT_EINVAL, "bad batch/domain index");
  *out = b->ctxs[d];
  return RMRT_OK;
}

int rmrt_batch_set_config(rmrt_batch* b, int cfg) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  if (cfg < 0 || cfg >= kNumTileShapes) return fail(RMRT_EINVAL, "config %d out of range", cfg);
  return batch_build_tiles(b, cfg, nullptr);
}

int rmrt_batch_step(rmrt_batch* b, int nsteps, void* stream) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(RMRT_EINVAL, "nsteps < 0");
  return batch_step_impl(b, nsteps, (hipStream_t)stream);
}

int rmrt_batch_step_prepare(rmrt_batch* b, int nsteps, void* stream) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(RMRT_EINVAL, "nsteps < 0");
  hipStream_t s = (hipStream_t)stream;
  hipGraphExec_t ge = nullptr;
  long long first = b->steps;
  int left = nsteps;
  while (left >= kGraphChunk) {
    int rc = batch_graph_for(b, kGraphChunk, first, &ge, s);
    if (rc != RMRT_OK) return rc;
    first += kGraphChunk;
    left -= kGraphChunk;
  }
  if (left > 1) return batch_graph_for(b, left, first, &ge, s);
  return RMRT_OK;
}

int rmrt_batch_autotune(rmrt_batch* b, int steps, void* stream, int* chosen) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  if (steps < 1) return fail(RMRT_EINVAL, "steps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.e0));
  HIP_TRY(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  int best = -1;
  float best_ms = 1e30f;
  for (int cfg = 0; cfg < kNumTileShapes; ++cfg) {
    int rc = batch_build_tiles(b, cfg, s);
    if (rc == RMRT_OK) rc = batch_step_impl(b, 2, s);  // warm-up (and graph capture)
    if (rc == RMRT_OK) rc = batch_step_impl(b, steps, s);  // captures the timed graph
    if (rc != RMRT_OK) return rc;
    HIP_TRY(hipEventRecord(e0, s));
    rc = batch_step_impl(b, steps, s);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    if (rc != RMRT_OK) return rc;
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = cfg;
    }
  }
  int rc = batch_build_tiles(b, best, s);
  if (rc != RMRT_OK) return rc;
  // then domain groups for the chosen shape: none, or groups of up to 128, 192
  // or 256 MiB of populations (the MALL holds 256 MB)
  const size_t group_cands[] = {0, (size_t)128 << 20, (size_t)192 << 20, (size_t)256 << 20};
  const size_t keep = b->group_bytes;
  size_t best_group = keep;
  best_ms = 1e30f;
  for (size_t gb : group_cands) {
    b->group_bytes = gb;
    batch_make_groups(b);
    rc = batch_step_impl(b, 2, s);
    if (rc == RMRT_OK) rc = batch_step_impl(b, steps, s);
    if (rc != RMRT_OK) return rc;
    HIP_TRY(hipEventRecord(e0, s));
    rc = batch_step_impl(b, steps, s);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    if (rc != RMRT_OK) return rc;
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best_group = gb;
    }
  }
  b->group_bytes = best_group;
  batch_make_groups(b);
  // then XCD chunks for the groups whose rows straddle cache lines, or none
  bool any_chunked = false;
  for (uint8_t g : b->group_chunked) any_chunked = any_chunked || g;
  if (any_chunked && !kTileShapes[best].persistent) {
    float mode_ms[2] = {0.f, 0.f};
    for (int mode = 0; mode < 2; ++mode) {
      b->xcd_chunks = mode;
      drop_graphs(b->graphs);
      rc = batch_step_impl(b, 2, s);
      if (rc == RMRT_OK) rc = batch_step_impl(b, steps, s);
      if (rc != RMRT_OK) return rc;
      HIP_TRY(hipEventRecord(e0, s));
      rc = batch_step_impl(b, steps, s);
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      if (rc != RMRT_OK) return rc;
      HIP_TRY(hipEventElapsedTime(&mode_ms[mode], e0, e1));
    }
    b->xcd_chunks = mode_ms[1] <= mode_ms[0] ? 1 : 0;
    drop_graphs(b->graphs);
  }
  if (chosen) *chosen = best;
  return RMRT_OK;
}

int rmrt_batch_set_xcd_chunks(rmrt_batch* b, int mode) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  if (mode != 0 && mode != 1) return fail(RMRT_EINVAL, "xcd chunk mode must be 0 or 1");
  b->xcd_chunks = mode;
  drop_graphs(b->graphs);
  return RMRT_OK;
}

int rmrt_batch_get_xcd_chunks(const rmrt_batch* b, int* mode, int* chunked_groups) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  if (mode) *mode = b->xcd_chunks;
  if (chunked_groups) {
    int n = 0;
    for (uint8_t g : b->group_chunked) n += g ? 1 : 0;
    *chunked_groups = n;
  }
  return RMRT_OK;
}

int rmrt_batch_set_group_bytes(rmrt_batch* b, size_t bytes) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  b->group_bytes = bytes;
  batch_make_groups(b);
  return RMRT_OK;
}

int rmrt_batch_get_group_bytes(const rmrt_batch* b, size_t* bytes, int* ngroups) {
  if (!b) return fail(RMRT_EINVAL, "batch is NULL");
  if (bytes) *bytes = b->group_bytes;
  if (ngroups) *ngroups = (int)b->groups.size();
  return RMRT_OK;
}

int rmrt_batch_residual(rmrt_batch* b, double* r, void* stream) {
  if (!b || !r) return fail(RMRT_EINVAL, "batch or r is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (!b->dres_all) HIP_TRY(hipMalloc(&b->dres_all, sizeof(double) * 2 * b->nd));
  if (!b->hres_all) HIP_TRY(hipHostMalloc(&b->hres_all, sizeof(double) * 2 * b->nd, hipHostMallocDefault));
  for (int d = 0; d < b->nd; ++d) {
    rmrt_ctx* c = b->ctxs[d];
    const int K = c->p.equation == RMRT_NSE ? c->v.d : 1;
    if (!c->uprev) HIP_TRY(hipMalloc(&c->uprev, sizeof(double) * (size_t)K * c->hdom.N));
    AuxLaunch a = aux_of(c, s);
    a.out0 = c->partials;
    a.out1 = c->uprev;
    a.flag = c->have_prev ? 1 : 0;
    hipError_t e = dispatch_residual(c->p.lattice, c->p.storage, a);
    if (e != hipSuccess) return fail(RMRT_EHIP, "residual launch: %s", hipGetErrorString(e));
    e = launch_reduce_final(c->partials, a.grid, b->dres_all + 2 * d, 2, s);
    if (e != hipSuccess) return fail(RMRT_EHIP, "residual final: %s", hipGetErrorString(e));
  }
  HIP_TRY(hipMemcpyAsync(b->hres_all, b->dres_all, sizeof(double) * 2 * b->nd, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int rc = RMRT_OK;
  for (int d = 0; d < b->nd; ++d) {
    rmrt_ctx* c = b->ctxs[d];
    const double num = b->hres_all[2 * d], den = b->hres_all[2 * d + 1];
    if (!c->have_prev) {
      r[d] = INFINITY;
    } else if (!std::isfinite(num) || !std::isfinite(den)) {
      r[d] = NAN;
      rc = fail(RMRT_ENONFINITE, "non-finite residual in domain %d", d);
    } else {
      r[d] = den > 0 ? std::sqrt(num / den) : (num > 0 ? INFINITY : 0.0);
    }
    c->have_prev = true;
  }
  return rc;
}

int rmrt_batch_free(rmrt_batch* b) {
  if (!b) return RMRT_OK;
  batch_release(b);
  delete b;
  return RMRT_OK;
}

}  // extern "C"
