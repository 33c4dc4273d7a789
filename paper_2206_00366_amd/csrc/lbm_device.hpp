// Device-side building blocks of the RMRT-LB step for gfx950.
//
// The collision works on raw moments (Sec. V eq. 5-2) of the stored
// deviations d_j = fbar_j - w_j rho0.  Because every lattice here is a subset
// of the 3^d tensor-product velocity set, M = D M~ (eq. Md2q9) factorises per
// axis: with the three populations (f-, f0, f+) of one lattice line,
//     (f- + f0 + f+,  f+ - f-,  f+ + f-)
// are the exponent-0/1/2 entries of M~ f, and the inverse is
//     f0 = mu0 - mu2,  f+- = (mu2 +- mu1) / 2.
// The kernel keeps the moments in that integer-matrix ("scaled") basis; the
// diagonal D is folded into host-side coefficient tables.  rD3Q19 runs the
// 27-slot transform with the 8 corner populations and the 8 moments with three
// non-zero exponents fixed at zero (those monomials vanish on rD3Q19, so the
// embedded inverse returns zero corners).  rD2Q5 and rD3Q7 run the 9- and
// 27-slot transforms in the same way, with every population slot and every
// moment that has two or more non-zero entries fixed at zero.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "lbm_params.hpp"

namespace rmrt {

// ----------------------------------------------------------------------------
// Lattices (paper velocity order; rD3Q27 edges j = 11..14 per the repaired
// x-z block of eq. 3-2b)
// ----------------------------------------------------------------------------
constexpr int kE27[27][3] = {
    {0, 0, 0},   {1, 0, 0},   {0, 1, 0},  {0, 0, 1},   {-1, 0, 0},  {0, -1, 0}, {0, 0, -1},
    {1, 1, 0},   {-1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {1, 0, 1},   {-1, 0, 1}, {-1, 0, -1},
    {1, 0, -1},  {0, 1, 1},   {0, -1, 1}, {0, -1, -1}, {0, 1, -1},  {1, 1, 1},  {1, 1, -1},
    {1, -1, 1},  {-1, 1, 1},  {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
constexpr int kE9[9][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                           {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};

template <int L>
struct Lat {
  static constexpr int D = (L == LAT_Q9 || L == LAT_Q5) ? 2 : 3;
  static constexpr int Q = L == LAT_Q9 ? 9 : L == LAT_Q19 ? 19 : L == LAT_Q27 ? 27 : L == LAT_Q5 ? 5 : 7;
  static constexpr int NS = (D == 2) ? 9 : 27;  // tensor slots
  // rD2Q5 / rD3Q7: NCDE with the linear equilibrium and the dB/dt term (eq. 4-16)
  static constexpr bool linear = (L == LAT_Q5 || L == LAT_Q7);
  static constexpr int e(int j, int a) { return (D == 2) ? kE9[j][a] : kE27[j][a]; }
  static constexpr int slot(int j) {
    return (e(j, 0) + 1) + 3 * (e(j, 1) + 1) + (D == 3 ? 9 * (e(j, 2) + 1) : 0);
  }
  // weight class of velocity j: 0 rest; 1, 2, 3 on the x, y, z axes; 4, 5, 6
  // in the xy, xz, yz planes; 7 corners
  static constexpr int wclass(int j) {
    const int x = e(j, 0) != 0, y = e(j, 1) != 0, z = e(j, 2) != 0;
    const int n = x + y + z;
    return n == 0 ? 0 : n == 3 ? 7 : n == 1 ? (x ? 1 : y ? 2 : 3) : (x && y ? 4 : x && z ? 5 : 6);
  }
  static constexpr int opp(int j) {
    for (int k = 0; k < Q; ++k)
      if (e(k, 0) == -e(j, 0) && e(k, 1) == -e(j, 1) && e(k, 2) == -e(j, 2)) return k;
    return -1;
  }
  static constexpr int nonzero_exps(int n) { return ((n % 3) != 0) + (((n / 3) % 3) != 0) + ((n / 9) != 0); }
  static constexpr int off_centre(int s) { return ((s % 3) != 1) + (((s / 3) % 3) != 1) + (D == 3 && (s / 9) != 1); }
  // moment slot that is not a moment of the lattice: three non-zero exponents
  // on rD3Q19, two or more on rD2Q5 / rD3Q7
  static constexpr bool dropped(int n) {
    return (L == LAT_Q19 && nonzero_exps(n) == 3) || (linear && nonzero_exps(n) >= 2);
  }
  // population slot not present in the lattice (rD3Q19 corners; rD2Q5 /
  // rD3Q7 everything off the axes)
  static constexpr bool absent(int s) {
    return (L == LAT_Q19 && off_centre(s) == 3) || (linear && off_centre(s) >= 2);
  }
  // the same as bit masks over the 3^D tensor slots
  static constexpr uint32_t absent_mask() {
    uint32_t m = 0;
    for (int s = 0; s < NS; ++s)
      if (absent(s)) m |= 1u << s;
    return m;
  }
  static constexpr uint32_t dropped_mask() {
    uint32_t m = 0;
    for (int n = 0; n < NS; ++n)
      if (dropped(n)) m |= 1u << n;
    return m;
  }
};

// Reciprocal in the working precision instead of the ~10-instruction IEEE
// division: the hardware v_rcp_f32 (1 ulp) for FP32, far below the FP32
// storage rounding; for FP64 v_rcp_f64 refined by two Newton steps
// r <- r + r (1 - x r), which squares the relative error each time and ends
// within an ulp or two of 1/x.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  return __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ----------------------------------------------------------------------------
// Storage: decode/encode of the stored deviations
// ----------------------------------------------------------------------------
template <int ST>
struct Store;
template <>
struct Store<ST_F64> {
  using S = double;
  using T = double;
  template <int J>
  __device__ static __forceinline__ T dec(S v, const Coef<T>&) { return v; }
  template <int J>
  __device__ static __forceinline__ S enc(T v, const Coef<T>&) { return v; }
};
template <>
struct Store<ST_F32> {
  using S = float;
  using T = float;
  template <int J>
  __device__ static __forceinline__ T dec(S v, const Coef<T>&) { return v; }
  template <int J>
  __device__ static __forceinline__ S enc(T v, const Coef<T>&) { return v; }
};
template <>
struct Store<ST_F16> {
  using S = _Float16;
  using T = float;
  // h_j = d_j / w_j keeps every slot well inside the normal half range; K is
  // the weight class of the velocity
  template <int K>
  __device__ static __forceinline__ T dec(S v, const Coef<T>& C) { return (float)v * C.wc[K]; }
  template <int K>
  __device__ static __forceinline__ S enc(T v, const Coef<T>& C) { return (_Float16)(v * C.iwc[K]); }
};

template <typename T>
__device__ __forceinline__ const Coef<T>& coef(const DomainDev& D);
template <>
__device__ __forceinline__ const Coef<double>& coef<double>(const DomainDev& D) { return D.cd; }
template <>
__device__ __forceinline__ const Coef<float>& coef<float>(const DomainDev& D) { return D.cf; }

// ----------------------------------------------------------------------------
// Per-axis factorised transforms on 3^D tensor slots.  Z is the mask of slots
// that are zero on entry (absent velocities before the forward transform,
// dropped monomials before the inverse); zeros are tracked through the axes
// so that no instruction adds a known zero (x + 0 cannot be folded by the
// compiler because of the sign of zero).
// ----------------------------------------------------------------------------
constexpr int axis_stride(int ax) { return ax == 0 ? 1 : (ax == 1 ? 3 : 9); }
constexpr bool zbit(uint32_t z, int s) { return (z >> s) & 1u; }

// zero mask after forward-transforming axis ax of a mask z
constexpr uint32_t fwd_zero_after(uint32_t z, int ax, int NS) {
  const int st = axis_stride(ax);
  uint32_t out = z;
  for (int b = 0; b < NS; ++b) {
    if ((b / st) % 3 != 0) continue;
    const bool zm = zbit(z, b), zz = zbit(z, b + st), zp = zbit(z, b + 2 * st);
    out &= ~((1u << b) | (1u << (b + st)) | (1u << (b + 2 * st)));
    if (zm && zz && zp) out |= 1u << b;
    if (zm && zp) out |= (1u << (b + st)) | (1u << (b + 2 * st));
  }
  return out;
}
constexpr uint32_t inv_zero_after(uint32_t z, int ax, int NS) {
  const int st = axis_stride(ax);
  uint32_t out = z;
  for (int b = 0; b < NS; ++b) {
    if ((b / st) % 3 != 0) continue;
    const bool z0 = zbit(z, b), z1 = zbit(z, b + st), z2 = zbit(z, b + 2 * st);
    out &= ~((1u << b) | (1u << (b + st)) | (1u << (b + 2 * st)));
    if (z1 && z2) out |= (1u << b) | (1u << (b + 2 * st));
    if (z0 && z2) out |= 1u << (b + st);
  }
  return out;
}
template <bool FWD>
constexpr uint32_t zero_before_axis(uint32_t z, int ax, int NS) {
  for (int a = 0; a < ax; ++a) z = FWD ? fwd_zero_after(z, a, NS) : inv_zero_after(z, a, NS);
  return z;
}

// (f-, f0, f+) -> (f- + f0 + f+, f+ - f-, f+ + f-) along each axis
template <int D, uint32_t Z, typename T, int NS>
__device__ __forceinline__ void moments_fwd(T (&t)[NS]) {
  static_for<0, D>([&](auto ax_) {
    constexpr int ax = decltype(ax_)::value;
    constexpr int st = axis_stride(ax);
    constexpr uint32_t z = zero_before_axis<true>(Z, ax, NS);
    static_for<0, NS>([&](auto b_) {
      constexpr int b = decltype(b_)::value;
      if constexpr ((b / st) % 3 == 0) {
        constexpr bool zm = zbit(z, b), zz = zbit(z, b + st), zp = zbit(z, b + 2 * st);
        const T m = t[b], c = t[b + st], p = t[b + 2 * st];
        T s, d;
        if constexpr (zm && zp) {
          s = T(0);
          d = T(0);
        } else if constexpr (zm) {
          s = p;
          d = p;
        } else if constexpr (zp) {
          s = m;
          d = -m;
        } else {
          s = m + p;
          d = p - m;
        }
        if constexpr (zm && zp)
          t[b] = c;
        else if constexpr (zz)
          t[b] = s;
        else
          t[b] = s + c;
        t[b + st] = d;
        t[b + 2 * st] = s;
      }
    });
  });
}

// (m0, m1, m2) -> ((m2 - m1)/2, m0 - m2, (m2 + m1)/2) along each axis
template <int D, uint32_t Z, typename T, int NS>
__device__ __forceinline__ void moments_inv(T (&t)[NS]) {
  static_for<0, D>([&](auto ax_) {
    constexpr int ax = decltype(ax_)::value;
    constexpr int st = axis_stride(ax);
    constexpr uint32_t z = zero_before_axis<false>(Z, ax, NS);
    static_for<0, NS>([&](auto b_) {
      constexpr int b = decltype(b_)::value;
      if constexpr ((b / st) % 3 == 0) {
        constexpr bool z0 = zbit(z, b), z1 = zbit(z, b + st), z2 = zbit(z, b + 2 * st);
        const T m0 = t[b], m1 = t[b + st], m2 = t[b + 2 * st];
        if constexpr (z1 && z2) {
          t[b] = T(0);
          t[b + 2 * st] = T(0);
        } else if constexpr (z1) {
          t[b] = T(0.5) * m2;
          t[b + 2 * st] = T(0.5) * m2;
        } else if constexpr (z2) {
          t[b] = T(-0.5) * m1;
          t[b + 2 * st] = T(0.5) * m1;
        } else {
          t[b] = T(0.5) * (m2 - m1);
          t[b + 2 * st] = T(0.5) * (m2 + m1);
        }
        if constexpr (z0 && z2)
          t[b + st] = T(0);
        else if constexpr (z2)
          t[b + st] = m0;
        else if constexpr (z0)
          t[b + st] = -m2;
        else
          t[b + st] = m0 - m2;
      }
    });
  });
}

// Central-moment shift (eq. 5-1-1) in the scaled basis: along each axis the
// line (m0, m1, m2) becomes (m0, m1 - v m0, m2 - 2 v m1 + v^2 m0) with
// v = u_a / c_a (the binomial shift of c_a^k m~_k by u_a), and back with -v.
template <int D, typename T, int NS>
__device__ __forceinline__ void central_shift(T (&t)[NS], const T (&v)[3]) {
  static_for<0, D>([&](auto ax_) {
    constexpr int ax = decltype(ax_)::value;
    constexpr int st = axis_stride(ax);
    const T w = v[ax];
    static_for<0, NS>([&](auto b_) {
      constexpr int b = decltype(b_)::value;
      if constexpr ((b / st) % 3 == 0) {
        const T m0 = t[b], m1 = t[b + st], m2 = t[b + 2 * st];
        t[b + st] = m1 - w * m0;
        t[b + 2 * st] = m2 - w * (T(2) * m1 - w * m0);
      }
    });
  });
}
template <int D, typename T, int NS>
__device__ __forceinline__ void central_unshift(T (&t)[NS], const T (&v)[3]) {
  static_for<0, D>([&](auto ax_) {
    constexpr int ax = decltype(ax_)::value;
    constexpr int st = axis_stride(ax);
    const T w = v[ax];
    static_for<0, NS>([&](auto b_) {
      constexpr int b = decltype(b_)::value;
      if constexpr ((b / st) % 3 == 0) {
        const T k0 = t[b], k1 = t[b + st], k2 = t[b + 2 * st];
        t[b + st] = k1 + w * k0;
        t[b + 2 * st] = k2 + w * (T(2) * k1 + w * k0);
      }
    });
  });
}

// Hermite-moment transform (eq. 5-1-1) in the scaled basis: along each axis the
// line (m0, m1, m2) becomes (m0, m1, m2 - th m0) with th = cs2 / c_a^2 (the
// tensor-product Hermite polynomials H_0 = 1, H_1 = xi, H_2 = xi^2 - cs2), and
// back with +th.  Lines whose second-order slot the lattice drops (rD3Q19's
// monomials with three non-zero exponents) are left alone: no kept slot
// depends on them.
template <int L, int D, typename T, int NS>
__device__ __forceinline__ void hermite_shift(T (&t)[NS], const T (&th)[3], T sign) {
  static_for<0, D>([&](auto ax_) {
    constexpr int ax = decltype(ax_)::value;
    constexpr int st = axis_stride(ax);
    const T w = sign * th[ax];
    static_for<0, NS>([&](auto b_) {
      constexpr int b = decltype(b_)::value;
      if constexpr ((b / st) % 3 == 0 && !Lat<L>::dropped(b + 2 * st)) t[b + 2 * st] -= w * t[b];
    });
  });
}

// Scaled raw moment n of g_eq(A, B, M) (eq. 3-3): only the terms that the
// lattice parity leaves non-zero are emitted.  Md = (Mxx, Myy, Mzz),
// Mo = (Mxy, Mxz, Myz).
template <int L, int n, typename T>
__device__ __forceinline__ T gmom(const Coef<T>& C, T A, const T (&B)[3], const T (&Md)[3],
                                  const T (&Mo)[3]) {
  constexpr int a = n % 3, b = (n / 3) % 3, p = n / 9;
  constexpr int nodd = (a & 1) + (b & 1) + (p & 1);
  if constexpr (Lat<L>::dropped(n)) {
    return T(0);
  } else if constexpr (nodd == 0) {
    T r = A * C.E0[n];
    if constexpr (!Lat<L>::linear) {   // the linear equilibrium has M = 0
      r += Md[0] * C.E2[n][0];
      r += Md[1] * C.E2[n][1];
      if constexpr (Lat<L>::D == 3) r += Md[2] * C.E2[n][2];
    }
    return r;
  } else if constexpr (nodd == 1) {
    constexpr int ax = (a & 1) ? 0 : ((b & 1) ? 1 : 2);
    return B[ax] * C.E1[n];
  } else if constexpr (nodd == 2) {
    constexpr int pr = (p & 1) == 0 ? 0 : ((a & 1) ? 1 : 2);  // xy, xz, yz
    return Mo[pr] * C.E3[n];
  } else {
    return T(0);
  }
}

// Source terms of one node: the parameter set's constants (F_CONST) or the
// node's field values (F_FIELD), in the form the collision uses (every term
// carries its factor dt; half_* are the half-step corrections of eq. 2-4).
// diff is dt/2 times the explicit difference S(t) - S(t - dt) of the gamma = 0
// NCDE form (eq. 2-1), zero otherwise.
template <typename T>
struct NodeSrc {
  T source, half_source, cs2_source, half_cs2_source, force[3], half_force[3], diff;
};
template <typename T>
__device__ __forceinline__ NodeSrc<T> const_sources(const Coef<T>& C) {
  NodeSrc<T> s;
  s.source = C.source;
  s.half_source = C.half_source;
  s.cs2_source = C.cs2_source;
  s.half_cs2_source = C.half_cs2_source;
  for (int a = 0; a < 3; ++a) {
    s.force[a] = C.force[a];
    s.half_force[a] = C.half_force[a];
  }
  s.diff = T(0);
  return s;
}
// from the node's source S, previous-step source Sp and body force F
template <typename T>
__device__ __forceinline__ NodeSrc<T> field_sources(const Coef<T>& C, T S, T Sp, const T (&F)[3]) {
  NodeSrc<T> s;
  s.source = C.dt * S;
  s.half_source = C.half_src_factor * S;
  s.cs2_source = C.dt_cs2 * S;
  s.half_cs2_source = C.half_dt_cs2 * S;
  for (int a = 0; a < 3; ++a) {
    s.force[a] = C.dt * F[a];
    s.half_force[a] = C.half_dt * F[a];
  }
  s.diff = C.half_dt * (S - Sp);
  return s;
}

// ----------------------------------------------------------------------------
// Collision of one node in deviation variables (eq. 2-2-3):
//   m* = m - S (m - m_eq') + (m_G + m_F),  m_eq' = m_eq - m_F / 2,
// with m_eq' = g_eq(rho - Sbar/2, rho u - Fbar/2, rho u u + cs2 Sbar I / 2)
// and m_G + m_F = g_eq(Sbar, Fbar, M_2G - cs2 Sbar I) for the NSE
// (eq. NSEfeq, NSEFeq, NSEGeq, M2GComput a), or
// m_eq' = g_eq(phi - S/2, phi u, phi u u), m_G + m_F = g_eq(S, M_1G, 0) with
// M_1G = (1 - s1/2) u S for the NCDE (eq. 4-14, 4-14-1, 4-11).  In the C = 0
// form (eq. 4-16: rD2Q5 / rD3Q7, or EQ_NCDE_C0) m_eq' = g_eq(phi - S/2, phi u, 0)
// and M_1G = (1 - s1/2) u (phi - phi_prev) / dt, with phi_prev the previous
// step's phi of the node; phi is returned in phi_out for the next step.  The
// gamma = 0 NCDE form adds dt (F(t) - F(t - dt)) / 2 = g_eq(src.diff, 0, 0).
// t[] holds the deviation populations in tensor slots on entry and the
// post-collision deviations on exit; src holds the node's source terms.
// ----------------------------------------------------------------------------
template <int L, int EQ, int FORCE, typename T, int NS>
__device__ __forceinline__ void collide(T (&t)[NS], const Coef<T>& C, const NodeSrc<T>& src,
                                        T phi_prev = T(0), T* phi_out = nullptr) {
  constexpr int D = Lat<L>::D;
  constexpr bool HIST = Lat<L>::linear || EQ == EQ_NCDE_C0;
  constexpr bool NSE = EQ == EQ_NSE || EQ == EQ_NSE_BASIS;
  // the central shift needs a moment set closed under it (rD2Q9, rD3Q27)
  constexpr bool CENTRAL_OK = L == LAT_Q9 || L == LAT_Q27;
  static_assert(EQ != EQ_NSE_BASIS || !Lat<L>::linear, "the basis collisions are NSE options");
  moments_fwd<D, Lat<L>::absent_mask()>(t);

  // slots of the first and second moments
  constexpr int sx = 1, sy = 3, sz = 9;
  constexpr int sxx = 2, syy = 6, szz = 18;
  const T drho = t[0];
  T m1[3];
  m1[0] = C.c[0] * t[sx];
  m1[1] = C.c[1] * t[sy];
  m1[2] = (D == 3) ? C.c[2] * t[sz] : T(0);

  T eA, eB[3], eMd[3], eMo[3];
  T sA = T(0), sB[3] = {T(0), T(0), T(0)}, sMd[3] = {T(0), T(0), T(0)}, sMo[3] = {T(0), T(0), T(0)};
  T s1 = T(0);
  T vc[3] = {T(0), T(0), T(0)};   // u_a / c_a of the central-moment shift
  if constexpr (NSE) {
    // eq. 2-4-2; without forcing the host guarantees Fbar = 0 and Sbar = 0, so
    // the kernel does not hold the half-step corrections at all
    const T rho = FORCE ? C.rho0 + drho + src.half_source : C.rho0 + drho;
    const T jx = FORCE ? m1[0] + src.half_force[0] : m1[0];
    const T jy = FORCE ? m1[1] + src.half_force[1] : m1[1];
    const T jz = FORCE ? m1[2] + src.half_force[2] : m1[2];
    // u = j / rho, or j / rho0 with the He-Luo equilibrium g_eq(rho, rho0 u, rho0 u u)
    const T ir = recip(C.hl ? C.rho0 : rho);
    const T ux = jx * ir, uy = jy * ir, uz = jz * ir;
    if constexpr (EQ == EQ_NSE_BASIS && CENTRAL_OK) {
      vc[0] = ux * C.inv_c[0];
      vc[1] = uy * C.inv_c[1];
      vc[2] = uz * C.inv_c[2];
    }
    eA = drho;
    eB[0] = m1[0];
    eB[1] = m1[1];
    eB[2] = m1[2];
    eMd[0] = jx * ux;
    eMd[1] = jy * uy;
    eMd[2] = jz * uz;
    eMo[0] = jx * uy;
    eMo[1] = jx * uz;
    eMo[2] = jy * uz;
    if constexpr (FORCE) {
      const T hs = src.half_cs2_source;
      eMd[0] += hs;
      eMd[1] += hs;
      eMd[2] += hs;
      // M_2G = (I - S2/2)(u F + F u + cs2 Sbar I)   (eq. M2GComput a)
      const T Txx = T(2) * ux * src.force[0] + src.cs2_source;
      const T Tyy = T(2) * uy * src.force[1] + src.cs2_source;
      const T Tzz = T(2) * uz * src.force[2] + src.cs2_source;
      sA = src.source;
      sB[0] = src.force[0];
      sB[1] = src.force[1];
      sB[2] = src.force[2];
      sMd[0] = C.IhS[0][0] * Txx + C.IhS[0][1] * Tyy + C.IhS[0][2] * Tzz - src.cs2_source;
      sMd[1] = C.IhS[1][0] * Txx + C.IhS[1][1] * Tyy + C.IhS[1][2] * Tzz - src.cs2_source;
      sMd[2] = C.IhS[2][0] * Txx + C.IhS[2][1] * Tyy + C.IhS[2][2] * Tzz - src.cs2_source;
      sMo[0] = C.ihs_off[0] * (ux * src.force[1] + uy * src.force[0]);
      sMo[1] = C.ihs_off[1] * (ux * src.force[2] + uz * src.force[0]);
      sMo[2] = C.ihs_off[2] * (uy * src.force[2] + uz * src.force[1]);
    }
  } else {
    const T phi = FORCE ? C.rho0 + drho + src.half_source : C.rho0 + drho;   // eq. 2-4-1
    const T Dphi = C.D0 * (T(1) + C.D2 * phi * phi);
    s1 = recip(T(0.5) + Dphi * C.inv_cs2_dt);                          // eq. 4-10
    eA = drho;
    eB[0] = phi * C.adv[0];
    eB[1] = phi * C.adv[1];
    eB[2] = phi * C.adv[2];
    if constexpr (HIST) {
      for (int k = 0; k < 3; ++k) eMd[k] = eMo[k] = T(0);
      if (phi_out) *phi_out = phi;
      if constexpr (FORCE) {
        // G from dB/dt = u (phi - phi_prev) / dt, first-order difference (eq. 4-16)
        const T g = (T(1) - T(0.5) * s1) * (phi - phi_prev) * C.inv_dt;
        sA = src.source;
        if constexpr (FORCE == F_FIELD) sA += src.diff;
        sB[0] = g * C.adv_g[0];
        sB[1] = g * C.adv_g[1];
        sB[2] = g * C.adv_g[2];
      }
    } else {
      // C = phi u u (adv_c = adv), or C = 0 at the diffusive scaling (adv_c = 0)
      eMd[0] = eB[0] * C.adv_c[0];
      eMd[1] = eB[1] * C.adv_c[1];
      eMd[2] = eB[2] * C.adv_c[2];
      eMo[0] = eB[0] * C.adv_c[1];
      eMo[1] = eB[0] * C.adv_c[2];
      eMo[2] = eB[1] * C.adv_c[2];
      if constexpr (FORCE) {
        const T g = (T(1) - T(0.5) * s1) * src.source;                  // eq. 4-11
        sA = src.source;
        if constexpr (FORCE == F_FIELD) sA += src.diff;
        sB[0] = g * C.adv_g[0];
        sB[1] = g * C.adv_g[1];
        sB[2] = g * C.adv_g[2];
      }
    }
  }

  if constexpr (EQ == EQ_NSE_BASIS) {
    // kappa* = kappa - Sbar (kappa - kappa_eq') + kappa_s with kappa = N m, N
    // the central shift N(u), the Hermite transform H or H N(u), or the BHLL
    // matrix, and the equilibrium and source moments transformed the same way
    // (eq. 5-1-2); Sbar has the raw model's blocks.  N is linear, so
    // m* = m - N^-1 Sbar N (m - eq') + src: only the non-equilibrium part d =
    // m - eq' goes into the basis and its relaxation comes back.  Conserved
    // moments of every basis are at their equilibrium (kappa_0 = rho', kappa_1 =
    // j - rho u = -dt F / 2 centrally), so only the source changes them.
    const bool cen = CENTRAL_OK && (C.basis & BASIS_CENTRAL);
    const bool her = (C.basis & BASIS_HERMITE) != 0;
    T d[NS];
    static_for<0, NS>([&](auto n_) {
      constexpr int n = decltype(n_)::value;
      d[n] = t[n] - gmom<L, n>(C, eA, eB, eMd, eMo);
    });
    bool bhll = false;
    if constexpr (L == LAT_Q9) bhll = (C.basis & BASIS_BHLL) != 0;
    if (bhll) {
      if constexpr (L == LAT_Q9) {
        // BHLL moments (eq. Md2q9-3) relaxed class by class: the host has formed
        // N^-1 Sbar_B N in this basis.  Its rows of the conserved moments vanish
        // and its columns there meet d = 0.  Non-conserved slot k: 2 (x^2), then
        // 4 .. 8.
        T nd6[6];
        static_for<0, 6>([&](auto k_) {
          constexpr int k = decltype(k_)::value;
          nd6[k] = d[k == 0 ? 2 : k + 3];
        });
        static_for<0, 6>([&](auto k_) {
          constexpr int k = decltype(k_)::value;
          T r = C.rb[k][0] * nd6[0];
          static_for<1, 6>([&](auto l_) {
            constexpr int l = decltype(l_)::value;
            r += C.rb[k][l] * nd6[l];
          });
          t[k == 0 ? 2 : k + 3] -= r;
        });
      }
    } else {
      if constexpr (CENTRAL_OK) {
        if (cen) central_shift<D>(d, vc);
      }
      if (her) hermite_shift<L, D>(d, C.hth, T(1));
      const T nd[3] = {d[sxx], d[syy], D == 3 ? d[szz] : T(0)};
      static_for<0, NS>([&](auto n_) {
        constexpr int n = decltype(n_)::value;
        constexpr int a = n % 3, b = (n / 3) % 3, p = n / 9;
        constexpr int ord = a + b + p;
        constexpr bool diag2 = (n == sxx || n == syy || n == szz);
        if constexpr (ord <= 1) {
          d[n] = T(0);
        } else if constexpr (diag2) {
          constexpr int ax = (n == sxx) ? 0 : (n == syy ? 1 : 2);
          T r = C.Sd[ax][0] * nd[0] + C.Sd[ax][1] * nd[1];
          if constexpr (D == 3) r += C.Sd[ax][2] * nd[2];
          d[n] = r;
        } else if constexpr (ord == 2) {
          constexpr int pr = (p == 0) ? 0 : ((a == 1) ? 1 : 2);
          d[n] *= C.s_off[pr];
        } else {
          d[n] *= C.s_hi;
        }
      });
      if (her) hermite_shift<L, D>(d, C.hth, T(-1));
      if constexpr (CENTRAL_OK) {
        if (cen) central_unshift<D>(d, vc);
      }
      static_for<0, NS>([&](auto n_) {
        constexpr int n = decltype(n_)::value;
        t[n] -= d[n];
      });
    }
    if constexpr (FORCE) {
      static_for<0, NS>([&](auto n_) {
        constexpr int n = decltype(n_)::value;
        t[n] += gmom<L, n>(C, sA, sB, sMd, sMo);
      });
    }
    moments_inv<D, Lat<L>::dropped_mask()>(t);
    return;
  }

  if constexpr (NSE) {
    // second-order diagonal block: full (D x D) relaxation matrix, scaled basis
    T nd[3];
    nd[0] = t[sxx] - gmom<L, sxx>(C, eA, eB, eMd, eMo);
    nd[1] = t[syy] - gmom<L, syy>(C, eA, eB, eMd, eMo);
    if constexpr (D == 3) nd[2] = t[szz] - gmom<L, szz>(C, eA, eB, eMd, eMo);
    T rx = C.Sd[0][0] * nd[0] + C.Sd[0][1] * nd[1];
    T ry = C.Sd[1][0] * nd[0] + C.Sd[1][1] * nd[1];
    T rz = T(0);
    if constexpr (D == 3) {
      rx += C.Sd[0][2] * nd[2];
      ry += C.Sd[1][2] * nd[2];
      rz = C.Sd[2][0] * nd[0] + C.Sd[2][1] * nd[1] + C.Sd[2][2] * nd[2];
    }
    t[sxx] -= rx;
    t[syy] -= ry;
    if constexpr (D == 3) t[szz] -= rz;
  }

  // Every other moment relaxes as m* = m - r (m - eq) + src.  g_eq is linear
  // in its arguments, so with eq = g_eq(e) and src = g_eq(s) this is
  // m* = (1 - r) m + g_eq(r e + s): one table evaluation per moment, with the
  // combined arguments formed once per rate.
  auto combine = [&](T r, T& cA, T (&cB)[3], T (&cMd)[3], T (&cMo)[3]) {
    cA = r * eA;
    for (int k = 0; k < 3; ++k) {
      cB[k] = r * eB[k];
      cMd[k] = r * eMd[k];
      cMo[k] = r * eMo[k];
    }
    if constexpr (FORCE) {
      cA += sA;
      for (int k = 0; k < 3; ++k) {
        cB[k] += sB[k];
        cMd[k] += sMd[k];
        cMo[k] += sMo[k];
      }
    }
  };
  T hA, hB[3], hMd[3], hMo[3];       // higher moments, rate s_hi
  combine(C.s_hi, hA, hB, hMd, hMo);
  const T keep_hi = T(1) - C.s_hi;

  static_for<0, NS>([&](auto n_) {
    constexpr int n = decltype(n_)::value;
    constexpr int a = n % 3, b = (n / 3) % 3, p = n / 9;
    constexpr int ord = a + b + p;
    constexpr bool diag2 = (n == sxx || n == syy || n == szz);
    if constexpr (Lat<L>::dropped(n)) {
      t[n] = T(0);
    } else if constexpr (ord == 0 || (NSE && (ord == 1 || diag2))) {
      // conserved (eq. 4-18-1), or NSE momentum (its rate is irrelevant), or
      // the diagonal second moments relaxed above: only the source is added
      if constexpr (FORCE) t[n] += gmom<L, n>(C, sA, sB, sMd, sMo);
    } else if constexpr (NSE && ord == 2) {
      constexpr int pr = (p == 0) ? 0 : ((a == 1) ? 1 : 2);
      T cA, cB[3], cMd[3], cMo[3];
      combine(C.s_off[pr], cA, cB, cMd, cMo);
      t[n] = (T(1) - C.s_off[pr]) * t[n] + gmom<L, n>(C, cA, cB, cMd, cMo);
    } else if constexpr (!NSE && ord == 1) {
      T cA, cB[3], cMd[3], cMo[3];
      combine(s1, cA, cB, cMd, cMo);
      t[n] = (T(1) - s1) * t[n] + gmom<L, n>(C, cA, cB, cMd, cMo);
    } else {
      t[n] = keep_hi * t[n] + gmom<L, n>(C, hA, hB, hMd, hMo);
    }
  });

  moments_inv<D, Lat<L>::dropped_mask()>(t);
}

}  // namespace rmrt
