// Kernels of the RMRT-LB step and its companions (init, macroscopic fields,
// FP64 reductions), templated over lattice, storage, equation, forcing,
// boundary handling and memory pattern.  Explicitly instantiated per
// (lattice, storage) in lbm_q*.hip.
//
// Memory patterns (stored state "natural" = slot j of node x holds f_j(x)):
//   PH_AB       read own slots of buffer `in`, write f*_j to slot j of x + e_j
//               in buffer `out` (push), or to slot opp(j) of x when x + e_j
//               is a wall or solid (halfway bounce-back).
//   PH_AA_EVEN  in place: read own slots, write f*_j to own slot opp(j).
//               Leaves the "swapped" state: f_j(x) sits in slot opp(j) of
//               x - e_j (or slot j of x when x - e_j bounces).
//   PH_AA_ODD   in place: read the swapped state, write like PH_AB.
// Every thread reads and writes the same address set in the AA patterns, so
// the in-place update has no races.
#pragma once

#include "lbm_device.hpp"

namespace rmrt {

#define RMRT_WALL_XM 1u
#define RMRT_WALL_XP 2u
#define RMRT_WALL_YM 4u
#define RMRT_WALL_YP 8u
#define RMRT_WALL_ZM 16u
#define RMRT_WALL_ZP 32u

// Buffers reach the kernels through the parameter block, so the compiler
// cannot see that they live in global memory; casting them to address space 1
// turns flat loads/stores (which also count against the LDS wait counter)
// into global ones.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* to_global(T* p) {
  return (gmem<T>*)p;
}
template <typename T>
__device__ __forceinline__ const gmem<T>* to_global(const T* p) {
  return (const gmem<T>*)p;
}

// Element i of one population stream (a per-lane 64-bit address: a scalar
// base plus 32-bit offset form needs 2 q live scalar registers per node and
// spills them).
template <typename T>
__device__ __forceinline__ T ld_elem(const gmem<T>* base, uint32_t i) { return base[i]; }
template <typename T>
__device__ __forceinline__ void st_elem(gmem<T>* base, uint32_t i, T v) { base[i] = v; }

// Buffer addressing of the population streams, for buffers below 4 GiB: a
// resource over the whole buffer, the stream start as the scalar byte offset
// and the node as the per-lane byte offset.  The scalar offsets are one
// 32-bit register per stream and the per-lane offset is shared by the q
// streams of a node, where the 64-bit form spends a pair of registers and an
// add per access.  num_records covers the buffer, so the per-lane offset is
// range checked by the hardware.
using BufRsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRawBufferWord3 = 0x00020000;   // gfx9 raw buffer: 32-bit data format
template <typename S>
__device__ __forceinline__ BufRsrc buf_rsrc(const gmem<S>* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(const S*)p, 0, (int)bytes, kRawBufferWord3);
}
// the resource a step kernel passes to its nodes: a buffer resource over the
// q streams with buffer addressing, an unused placeholder without (which
// leaves the 64-bit form's code exactly as it is without this option)
template <bool BUF>
struct StreamRes {
  using type = int;
  template <int Q, typename S>
  __device__ static __forceinline__ type make(const gmem<S>*, uint32_t) { return 0; }
};
template <>
struct StreamRes<true> {
  using type = BufRsrc;
  template <int Q, typename S>
  __device__ static __forceinline__ type make(const gmem<S>* p, uint32_t ld) {
    return buf_rsrc(p, (uint32_t)Q * ld * (uint32_t)sizeof(S));
  }
};
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename S>
__device__ __forceinline__ S buf_ld(BufRsrc r, uint32_t lane_off, uint32_t stream_off) {
  if constexpr (sizeof(S) == 2)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, lane_off, stream_off, 0));
  else if constexpr (sizeof(S) == 4)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, stream_off, 0));
  else
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, stream_off, 0));
}
template <typename S>
__device__ __forceinline__ void buf_st(BufRsrc r, uint32_t lane_off, uint32_t stream_off, S v) {
  if constexpr (sizeof(S) == 2)
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, lane_off, stream_off, 0);
  else if constexpr (sizeof(S) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, lane_off, stream_off, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, lane_off, stream_off, 0);
}

// exact n / d for n < 2^32 with m = floor(2^32 / d) (0xffffffff for d = 1)
__device__ __forceinline__ uint32_t fast_div(uint32_t n, uint32_t d, uint32_t m, uint32_t& r) {
  uint32_t q = __umulhi(n, m);
  uint32_t rr = n - q * d;
  if (rr >= d) {
    q += 1;
    rr -= d;
  }
  r = rr;
  return q;
}

// Geometry of one node: neighbour offsets with periodic wrap and wall flags.
#ifndef RMRT_CHECKED
#define RMRT_CHECKED 0
#endif
// Neighbour node index n of node self.  The checked build (RMRT_CHECKED = 1,
// librmrt_checked.so) tests it against Dm.oob_limit, counts an index outside
// it in *Dm.oob and takes the node's own index instead, so that the access
// stays inside the buffers; the production build compiles the test away.
__device__ __forceinline__ uint32_t checked_node(const DomainDev& Dm, uint32_t n, uint32_t self) {
  if constexpr (RMRT_CHECKED != 0) {
    if (n >= Dm.oob_limit) {
      atomicAdd(Dm.oob, 1u);
      return self < Dm.oob_limit ? self : 0u;
    }
  }
  return n;
}

template <int D>
struct Geo {
  int32_t ox[3], oy[3], oz[3];
  bool lo[3], hi[3];
  __device__ __forceinline__ void make(const DomainDev& Dm, uint32_t idx) {
    uint32_t x, y, z, r;
    const uint32_t q1 = fast_div(idx, Dm.nx, Dm.mnx, r);
    x = r;
    if constexpr (D == 2) {
      y = q1;
      z = 0;
    } else {
      z = fast_div(idx, Dm.nxny, Dm.mnxny, r);
      y = q1 - z * Dm.ny;
    }
    const int32_t nx = (int32_t)Dm.nx, ny = (int32_t)Dm.ny, nz = (int32_t)Dm.nz;
    const int32_t nxny = (int32_t)Dm.nxny;
    ox[0] = (x == 0) ? nx - 1 : -1;
    ox[1] = 0;
    ox[2] = (x == Dm.nx - 1) ? 1 - nx : 1;
    oy[0] = (y == 0) ? (ny - 1) * nx : -nx;
    oy[1] = 0;
    oy[2] = (y == Dm.ny - 1) ? -(ny - 1) * nx : nx;
    if constexpr (D == 3) {
      oz[0] = (z == 0) ? (nz - 1) * nxny : -nxny;
      oz[2] = (z == Dm.nz - 1) ? -(nz - 1) * nxny : nxny;
    } else {
      oz[0] = 0;
      oz[2] = 0;
    }
    oz[1] = 0;
    const uint32_t w = Dm.walls;
    lo[0] = (x == 0) && (w & RMRT_WALL_XM);
    hi[0] = (x == Dm.nx - 1) && (w & RMRT_WALL_XP);
    lo[1] = (y == 0) && (w & RMRT_WALL_YM);
    hi[1] = (y == Dm.ny - 1) && (w & RMRT_WALL_YP);
    lo[2] = (D == 3) && (z == 0) && (w & RMRT_WALL_ZM);
    hi[2] = (D == 3) && (z == Dm.nz - 1) && (w & RMRT_WALL_ZP);
  }
  template <int L, int J>
  __device__ __forceinline__ int32_t off() const {
    constexpr int ex = Lat<L>::e(J, 0), ey = Lat<L>::e(J, 1), ez = Lat<L>::e(J, 2);
    return ox[ex + 1] + oy[ey + 1] + oz[ez + 1];
  }
  // the neighbour of node idx along e_J (periodic wrap included)
  template <int L, int J>
  __device__ __forceinline__ uint32_t nbr(const DomainDev& Dm, uint32_t idx) const {
    return checked_node(Dm, (uint32_t)(idx + (uint32_t)off<L, J>()), idx);
  }
  // does the link from this node along e_J hit a wall face (or, with SOLID, a
  // solid node of the byte mask)?
  template <int L, int J, bool SOLID = true>
  __device__ __forceinline__ bool bounce(const DomainDev& Dm, uint32_t idx) const {
    constexpr int ex = Lat<L>::e(J, 0), ey = Lat<L>::e(J, 1), ez = Lat<L>::e(J, 2);
    if constexpr (ex == 0 && ey == 0 && ez == 0) return false;
    bool b = false;
    if constexpr (ex < 0) b = b || lo[0];
    if constexpr (ex > 0) b = b || hi[0];
    if constexpr (ey < 0) b = b || lo[1];
    if constexpr (ey > 0) b = b || hi[1];
    if constexpr (ez < 0) b = b || lo[2];
    if constexpr (ez > 0) b = b || hi[2];
    if constexpr (SOLID)
      if (Dm.has_solid) b = b || (to_global(Dm.solid)[nbr<L, J>(Dm, idx)] != 0);
    return b;
  }
};

// Per-node link bits of the solid-mask boundary mode (BC == 2): built once by
// k_links from the walls and the solid mask, so the step reads one word per
// node instead of a byte per neighbour.
template <int L>
struct LinkBits {
  using W = typename std::conditional<(Lat<L>::Q <= 15), uint16_t, uint32_t>::type;
  static constexpr W kSolid = (W)1 << (sizeof(W) * 8 - 1);
};

// Element offset (in S units, from the buffer start) of the slot read for
// population j of node idx, in the natural (own) or swapped layout.
template <int L, int BC, bool SWAPPED, int J, int D>
__device__ __forceinline__ size_t read_elem(const DomainDev& Dm, const Geo<D>& g, uint32_t idx) {
  const size_t LD = Dm.ld;
  if constexpr (!SWAPPED) {
    return (size_t)J * LD + idx;
  } else {
    constexpr int O = Lat<L>::opp(J);
    if constexpr (BC == 1) {
      if (g.template bounce<L, O>(Dm, idx)) return (size_t)J * LD + idx;
    }
    return (size_t)O * LD + g.template nbr<L, O>(Dm, idx);
  }
}

// ----------------------------------------------------------------------------
// The fused collide-and-stream kernel.  Work is a list of tiles (contiguous
// node ranges of a domain); a null tile list means one domain split into
// tiles of `tile_nodes` nodes with one tile per workgroup.
// ----------------------------------------------------------------------------
// kinds of local output (stress / strain rate of the NSE, grad phi of the NCDE)
enum { GRAD_STRAIN = 0, GRAD_STRESS = 1, GRAD_PHI = 2 };

// The local outputs of one node from its deviations d_j (paper order), in the
// working precision T: FP64 in the on-demand kernel, the step's precision in
// the fused step.  prev: phi of the previous step (rD2Q5 / rD3Q7).
template <int L, int EQ, typename T>
__device__ __forceinline__ void local_node(const DomainDev& Dm, const Coef<T>& C, const T (&d)[Lat<L>::Q], T prev,
                                           int kind, T (&res)[6]) {
  constexpr int D = Lat<L>::D;
  T drho = T(0), m1[3] = {T(0), T(0), T(0)};
  static_for<0, Lat<L>::Q>([&](auto j_) {
    constexpr int J = decltype(j_)::value;
    drho += d[J];
    if constexpr (Lat<L>::e(J, 0) != 0) m1[0] += (T)Lat<L>::e(J, 0) * d[J];
    if constexpr (Lat<L>::e(J, 1) != 0) m1[1] += (T)Lat<L>::e(J, 1) * d[J];
    if constexpr (Lat<L>::e(J, 2) != 0) m1[2] += (T)Lat<L>::e(J, 2) * d[J];
  });
  m1[0] *= C.c[0];
  m1[1] *= C.c[1];
  m1[2] *= C.c[2];
  const T r = C.rho0 + drho + C.half_source;
  if constexpr (EQ == EQ_NSE) {
    // second moments of the deviations: sum c_a c_b d_j (the rest part
    // w_j rho0 contributes rho0 cs2 I)
    T m2[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
    static_for<0, Lat<L>::Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      constexpr int e0 = Lat<L>::e(J, 0), e1 = Lat<L>::e(J, 1), e2 = Lat<L>::e(J, 2);
      if constexpr (e0 != 0) m2[0][0] += d[J];
      if constexpr (e1 != 0) m2[1][1] += d[J];
      if constexpr (e2 != 0) m2[2][2] += d[J];
      if constexpr (e0 * e1 != 0) m2[0][1] += (T)(e0 * e1) * d[J];
      if constexpr (e0 * e2 != 0) m2[0][2] += (T)(e0 * e2) * d[J];
      if constexpr (e1 * e2 != 0) m2[1][2] += (T)(e1 * e2) * d[J];
    });
    const T ru = C.hl ? C.rho0 : r;   // He-Luo: f_eq = g_eq(rho, rho0 u, rho0 u u)
    const T ir = recip(ru);
    T u[3];
    for (int a = 0; a < 3; ++a) u[a] = (m1[a] + C.half_force[a]) * ir;
    // v = m_2^ne + dt/2 (u F + F u + (cs2 I - u u) S) on the 2nd-order rows
    T v[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const T m2ab = (a <= b ? m2[a][b] : m2[b][a]) * C.c[a] * C.c[b] + (a == b ? C.rho0 * C.cs2 : T(0));
        v[a][b] = m2ab - (a == b ? r * C.cs2 : T(0)) - ru * u[a] * u[b] + u[a] * C.half_force[b] +
                  C.half_force[a] * u[b] + (a == b ? C.half_cs2_source : T(0)) - u[a] * u[b] * C.half_source;
      }
    T tau[3][3];
    for (int a = 0; a < 3; ++a) {
      T sum = T(0);
      for (int b = 0; b < D; ++b) sum += C.IhS[a][b] * v[b][b];
      tau[a][a] = -sum;
    }
    tau[0][1] = -C.ihs_off[0] * v[0][1];
    tau[0][2] = -C.ihs_off[1] * v[0][2];
    tau[1][2] = -C.ihs_off[2] * v[1][2];
    T o[3][3];
    if (kind == GRAD_STRESS) {
      for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) o[a][b] = tau[a][b];
    } else {
      // eq. 4-28 with the tensors of eq. 4-29: tau_ab = 2 K_ab E_ab (a != b),
      // tau_aa = K_aa (2 E_aa - (2/d) tr E) + Kb_a tr E, K = rho nu_entry.
      // Summing tau_aa / (2 K_aa) gives tr E (1 + sum_a (Kb_a - 2 K_aa / d) /
      // (2 K_aa)), whose factor is rho-free and precomputed.
      const InitCoef& I = Dm.ic;
      T num = T(0);
      for (int a = 0; a < D; ++a) num += tau[a][a] * (T)I.inv2nu_diag[a];
      const T trE = num * ir * (T)I.inv_trace_den;
      for (int a = 0; a < 3; ++a) o[a][a] = T(0);
      for (int a = 0; a < D; ++a)
        o[a][a] = (tau[a][a] - ru * (T)I.bulk_excess[a] * trE) * ir * (T)I.inv2nu_diag[a];
      o[0][1] = tau[0][1] * ir * (T)I.inv2nu_pair[0];
      o[0][2] = tau[0][2] * ir * (T)I.inv2nu_pair[1];
      o[1][2] = tau[1][2] * ir * (T)I.inv2nu_pair[2];
    }
    res[0] = o[0][0];
    res[1] = o[1][1];
    if constexpr (D == 2) {
      res[2] = o[0][1];
    } else {
      res[2] = o[2][2];
      res[3] = o[0][1];
      res[4] = o[0][2];
      res[5] = o[1][2];
    }
  } else {
    const T Dphi = C.D0 * (T(1) + C.D2 * r * r);
    const T s1 = recip(T(0.5) + Dphi * C.inv_cs2_dt);
    const T iD = recip(Dphi);
    T X = C.source;
    if (C.hist_g) X = (r - prev) * C.inv_dt;   // C = 0 form: dB/dt = u (phi - phi_prev) / dt
    for (int a = 0; a < D; ++a)
      res[a] = -(T(1) - T(0.5) * s1) * (m1[a] - r * C.adv[a] + T(0.5) * C.dt * C.adv_g[a] * X) * iD;
  }
}

// BUF: buffer addressing (buffers below 4 GiB).  FORCE: F_NONE, F_CONST or
// F_FIELD (the node's source terms read from the domain's field arrays).
template <int L, int ST, int EQ, int FORCE, int BC, int PH, bool BUF>
struct NodeStep {
  using R = typename StreamRes<BUF>::type;
  using SS = Store<ST>;
  using S = typename SS::S;
  using T = typename SS::T;
  using LW = typename LinkBits<L>::W;
  static constexpr int Q = Lat<L>::Q, NS = Lat<L>::NS, D = Lat<L>::D;
  static constexpr bool HIST = Lat<L>::linear || EQ == EQ_NCDE_C0;   // C = 0 form: previous phi

  T t[NS];
  Geo<D> g;
  LW lb;
  uint32_t idx;
  bool live;   // a fluid node to update
  bool edge;   // buffer addressing with walls: some lane of the wave has a bounced link
  T phi_prev;  // C = 0 form: phi of the previous step
  T src_s;     // F_FIELD: the node's source S (kept for the gamma = 0 previous-step field)
  NodeSrc<T> src;

  // Boundary modes: 0 periodic; 1 wall faces from the coordinates (the host
  // never pairs it with a solid mask: a mask selects mode 2); 2 link words.
  // Bounced links pick their address with a select, not a branch, so the
  // wave's q loads and stores stay back to back.  With buffer addressing a
  // wave none of whose nodes has a bounced link takes the periodic addresses
  // (scalar stream offset); the other waves select full 32-bit offsets.

  // does link J of this node bounce?
  template <int J>
  __device__ __forceinline__ bool bounced(const DomainDev& Dm) const {
    if constexpr (BC == 2)
      return (lb >> J) & 1;
    else
      return g.template bounce<L, J, false>(Dm, idx);
  }

  // Read the q populations of node idx_ (nothing for solid or invalid nodes).
  __device__ __forceinline__ void load(const DomainDev& Dm, const Coef<T>& C, const gmem<S>* fin, R rin,
                                       uint32_t idx_, bool valid) {
    idx = valid ? checked_node(Dm, idx_, 0u) : idx_;
    live = valid;
    lb = 0;
    if constexpr (BC == 2) {
      if (live) {
        lb = to_global((const LW*)Dm.links)[idx];
        if (lb & LinkBits<L>::kSolid) live = false;
      }
    }
    if (!live) return;
    if constexpr (HIST) phi_prev = to_global((const T*)Dm.hist)[idx];
    if constexpr (FORCE == F_FIELD) {
      // field values of this node (null arrays are zero; every node of a
      // domain takes the same branch)
      const T Sn = Dm.src ? to_global((const T*)Dm.src)[idx] : T(0);
      T F[3] = {T(0), T(0), T(0)};
      if constexpr (EQ == EQ_NSE || EQ == EQ_NSE_BASIS) {
        if (Dm.frc)
          for (int a = 0; a < D; ++a) F[a] = to_global((const T*)Dm.frc)[(size_t)a * Dm.N + idx];
      }
      const T Sp = Dm.sprev ? to_global((const T*)Dm.sprev)[idx] : Sn;
      src_s = Sn;
      src = field_sources<T>(C, Sn, Sp, F);
    } else {
      src = const_sources<T>(C);
    }
    if constexpr (PH != PH_AA_EVEN) g.make(Dm, idx);
    edge = false;
    if constexpr (BUF && BC != 0 && PH != PH_AA_EVEN) {
      bool e;
      if constexpr (BC == 2)
        e = (lb & (LW)~LinkBits<L>::kSolid) != 0;
      else
        e = g.lo[0] | g.hi[0] | g.lo[1] | g.hi[1] | g.lo[2] | g.hi[2];
      edge = __builtin_amdgcn_ballot_w64(e) != 0;   // wave-uniform
    }
    const uint32_t LD = Dm.ld;   // stream stride
    static_for<0, NS>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      if constexpr (Lat<L>::absent(s)) t[s] = T(0);
    });
    if constexpr (BUF && BC != 0 && PH == PH_AA_ODD) {
      if (edge)
        load_buf<true>(C, Dm, rin, LD);
      else
        load_buf<false>(C, Dm, rin, LD);
      return;
    }
    static_for<0, Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      S v;
      if constexpr (BUF) {
        constexpr int O = Lat<L>::opp(J);
        constexpr uint32_t es = sizeof(S);
        if constexpr (PH == PH_AA_ODD)
          v = buf_ld<S>(rin, g.template nbr<L, O>(Dm, idx) * es, (uint32_t)O * LD * es);
        else
          v = buf_ld<S>(rin, idx * es, (uint32_t)J * LD * es);
      } else if constexpr (PH == PH_AA_ODD) {
        // swapped layout: the value for direction J sits in slot O of the
        // upstream node, or in this node's own slot J when that link bounced
        constexpr int O = Lat<L>::opp(J);
        const gmem<S>* pu = fin + (size_t)O * LD + g.template nbr<L, O>(Dm, idx);
        if constexpr (BC == 0) {
          v = *pu;
        } else {
          bool b;
          if constexpr (BC == 2)
            b = (lb >> O) & 1;
          else
            b = g.template bounce<L, O, false>(Dm, idx);
          const gmem<S>* po = fin + (size_t)J * LD + idx;
          v = *(b ? po : pu);
        }
      } else {
        v = ld_elem(fin + (size_t)J * LD, idx);
      }
      t[Lat<L>::slot(J)] = SS::template dec<Lat<L>::wclass(J)>(v, C);
    });
  }

  // Odd AA phase with walls and buffer addressing: EDGE selects, per link,
  // this node's own slot J (bounced) or slot O of the upstream node.
  template <bool EDGE>
  __device__ __forceinline__ void load_buf(const Coef<T>& C, const DomainDev& Dm, R rin, uint32_t LD) {
    static_for<0, Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      constexpr int O = Lat<L>::opp(J);
      constexpr uint32_t es = sizeof(S);
      const uint32_t up = g.template nbr<L, O>(Dm, idx);
      S v;
      if constexpr (EDGE) {
        const uint32_t full = bounced<O>(Dm) ? (uint32_t)J * LD + idx : (uint32_t)O * LD + up;
        v = buf_ld<S>(rin, full * es, 0u);
      } else {
        v = buf_ld<S>(rin, up * es, (uint32_t)O * LD * es);
      }
      t[Lat<L>::slot(J)] = SS::template dec<Lat<L>::wclass(J)>(v, C);
    });
  }

  // Pushing stores with walls and buffer addressing (odd AA phase, AB).
  template <bool EDGE>
  __device__ __forceinline__ void store_buf(const Coef<T>& C, const DomainDev& Dm, R rout, uint32_t LD) {
    static_for<0, Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      constexpr int O = Lat<L>::opp(J);
      constexpr uint32_t es = sizeof(S);
      const S v = SS::template enc<Lat<L>::wclass(J)>(t[Lat<L>::slot(J)], C);
      const uint32_t down = g.template nbr<L, J>(Dm, idx);
      if constexpr (EDGE) {
        const uint32_t full = bounced<J>(Dm) ? (uint32_t)O * LD + idx : (uint32_t)J * LD + down;
        buf_st<S>(rout, full * es, 0u, v);
      } else {
        buf_st<S>(rout, down * es, (uint32_t)J * LD * es, v);
      }
    });
  }

  // Local outputs of the state this node's update starts from (the loaded
  // deviations, before the collision), in the working precision; zero at
  // solid nodes.  Component k of node idx at out[k N + idx].
  __device__ __forceinline__ void local_out(const DomainDev& Dm, const Coef<T>& C, void* out, int kind,
                                            int out_f32) const {
    constexpr int NC = (EQ == EQ_NSE) ? D * (D + 1) / 2 : D;
    T res[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (live) {
      T d[Q];
      static_for<0, Q>([&](auto j_) {
        constexpr int J = decltype(j_)::value;
        d[J] = t[Lat<L>::slot(J)];
      });
      T prev = T(0);
      if constexpr (HIST) prev = phi_prev;
      local_node<L, (EQ == EQ_NSE ? EQ_NSE : EQ_NCDE), T>(Dm, C, d, prev, kind, res);
    }
    const size_t N = Dm.N;
    for (int k = 0; k < NC; ++k) {
      if (out_f32)
        to_global((float*)out)[(size_t)k * N + idx] = (float)res[k];
      else
        to_global((double*)out)[(size_t)k * N + idx] = (double)res[k];
    }
  }

  // Collide and write the q post-collision populations.
  __device__ __forceinline__ void finish(const DomainDev& Dm, const Coef<T>& C, gmem<S>* fout, R rout) {
    if (!live) return;
    if constexpr (HIST) {
      T phi;
      collide<L, EQ, FORCE>(t, C, src, phi_prev, &phi);
      to_global((T*)Dm.hist)[idx] = phi;
    } else {
      collide<L, EQ, FORCE>(t, C, src);
    }
    if constexpr (FORCE == F_FIELD) {
      if (Dm.sprev) to_global((T*)Dm.sprev)[idx] = src_s;   // F(t - dt) of the next step
    }
    // Stream stride.  Under FP32 and FP16 storage on rD2Q9 / rD3Q19 / rD3Q27 it
    // is taken here as a new value (readfirstlane, then an empty asm the compiler
    // must treat as changing it), so that the store offsets J * LD are formed
    // after the collision instead of being held in scalar registers across it:
    // that removes most of the scalar-register spills of the odd step (rD3Q19
    // FP32: 62 to 16 lane reads) and made rD3Q19 / rD3Q27 FP32 steps 1.4-2%
    // faster; the FP64 steps and the linear lattices ran 1-2.5% slower with it.
    uint32_t LD = Dm.ld;
    if constexpr (ST != ST_F64 && !Lat<L>::linear) {
      LD = __builtin_amdgcn_readfirstlane(LD);
      asm volatile("" : "+s"(LD));
    }
    if constexpr (BUF && BC != 0 && PH != PH_AA_EVEN) {
      if (edge)
        store_buf<true>(C, Dm, rout, LD);
      else
        store_buf<false>(C, Dm, rout, LD);
      return;
    }
    static_for<0, Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      constexpr int O = Lat<L>::opp(J);
      const S v = SS::template enc<Lat<L>::wclass(J)>(t[Lat<L>::slot(J)], C);
      constexpr uint32_t es = sizeof(S);
      if constexpr (BUF && PH == PH_AA_EVEN) {
        buf_st<S>(rout, idx * es, (uint32_t)O * LD * es, v);
      } else if constexpr (BUF) {
        buf_st<S>(rout, g.template nbr<L, J>(Dm, idx) * es, (uint32_t)J * LD * es, v);
      } else if constexpr (PH == PH_AA_EVEN) {
        st_elem(fout + (size_t)O * LD, idx, v);
      } else if constexpr (BC == 0) {
        st_elem(fout + (size_t)J * LD, g.template nbr<L, J>(Dm, idx), v);
      } else {
        bool b;
        if constexpr (BC == 2)
          b = (lb >> J) & 1;
        else
          b = g.template bounce<L, J, false>(Dm, idx);
        gmem<S>* pd = fout + (size_t)J * LD + g.template nbr<L, J>(Dm, idx);
        gmem<S>* pb = fout + (size_t)O * LD + idx;
        *(b ? pb : pd) = v;
      }
    });
  }
};

// Tile order.  Workgroups are dealt round-robin to the 8 XCDs.  With
// STEP_XCD_ORDER each XCD takes a contiguous range of the tile list instead, so
// that neighbouring tiles share its L2: with one workgroup per tile (gridDim ==
// ntiles) workgroup b of XCD b % 8 takes tile b / 8 of that XCD's range; with a
// persistent grid (gridDim < ntiles, a multiple of 8 when XCD_ORDER is set)
// each XCD walks its own contiguous eighth of the list.  The grid size is the
// occupancy knob (fewer resident waves keep the q concurrent address streams
// per wave from oversubscribing HBM).
// STEP_ALTERNATE_ORDER walks the tiles backwards on odd steps, so that each
// step starts on the tiles the previous one finished with, whose data the
// memory-side cache (MALL) and the L2 still hold.
// STEP_XCD_CHUNKS (one workgroup per tile only; odd AA and AB steps) deals
// runs of kXcdChunk consecutive tiles to one XCD, the eight XCDs' runs
// interleaved: the chip still sweeps the list in order, and only one tile
// boundary in kXcdChunk lies between two XCDs' L2s.  The odd AA step (and the
// AB step's pushes) read and write cache lines that straddle tile boundaries
// whenever a neighbour offset is not a whole number of lines (rows of
// nx % 32 != 0 nodes in FP32); a line written in part by two XCDs reaches
// memory as two partial writes.  The even AA step touches only its own
// nodes' slots and keeps the plain round-robin order.
enum : uint32_t {
  STEP_XCD_ORDER = 1u,
  STEP_PERSISTENT = 2u,
  STEP_WIDE_TILES = 4u,
  STEP_BUFFER_OFFSETS = 8u,
  STEP_ALTERNATE_ORDER = 16u,
  STEP_XCD_CHUNKS = 32u
};
constexpr uint32_t kXcdChunk = 16;

// Tile of workgroup b (on XCD b % 8) under STEP_XCD_CHUNKS; the ragged end of
// the list (fewer than 8 kXcdChunk tiles) keeps the identity, so the map is a
// bijection of [0, ntiles).
__device__ __forceinline__ uint32_t xcd_chunk_tile(uint32_t b, uint32_t ntiles) {
  constexpr uint32_t M = 8u * kXcdChunk;
  const uint32_t full = ntiles / M * M;
  if (b >= full) return b;
  const uint32_t x = b & 7u, l = b >> 3;
  return (l / kXcdChunk) * M + x * kXcdChunk + (l % kXcdChunk);
}

// NPT nodes per thread per pass (1, or 2 with tiles of 2 blockDim nodes: both
// nodes are read before either collides, so each wave keeps 2 q loads in
// flight).  BUF selects buffer addressing of the population streams (the host
// sets it only where every population buffer is below 4 GiB).
template <int L, int ST, int EQ, int FORCE, int BC, int PH, int NPT, bool BUF>
__global__ void __launch_bounds__(256)
    k_step(const DomainDev* __restrict__ doms, const Tile* __restrict__ tiles, uint32_t ntiles,
           uint32_t tile_nodes, uint32_t parity, uint32_t flags) {
  using SS = Store<ST>;
  using S = typename SS::S;
  using T = typename SS::T;
  const uint32_t G = gridDim.x;
  const bool xcd = (flags & STEP_XCD_ORDER) != 0;
  // odd steps of the alternating order walk backwards; with the XCD order each
  // XCD reverses its own range, so that it keeps the tiles its L2 holds
  const bool rev = (flags & STEP_ALTERNATE_ORDER) && (parity & 1u);
  const uint32_t per = (ntiles + 7u) >> 3;
  for (uint32_t it = 0;; ++it) {
    uint32_t tt;
    if (G >= ntiles) {
      if (it > 0 || blockIdx.x >= ntiles) break;
      if (xcd) {
        const uint32_t x = blockIdx.x & 7u, local = blockIdx.x >> 3;
        const uint32_t q8 = ntiles >> 3, rem = ntiles & 7u;
        const uint32_t first = x * q8 + (x < rem ? x : rem), cnt = q8 + (x < rem ? 1u : 0u);
        tt = first + (rev ? cnt - 1u - local : local);
      } else if (PH != PH_AA_EVEN && (flags & STEP_XCD_CHUNKS)) {
        tt = xcd_chunk_tile(blockIdx.x, ntiles);
        if (rev) tt = ntiles - 1u - tt;
      } else {
        tt = rev ? ntiles - 1u - blockIdx.x : blockIdx.x;
      }
    } else if (xcd) {
      const uint32_t local = (blockIdx.x >> 3) + it * (G >> 3);
      const uint32_t first = (blockIdx.x & 7u) * per;
      const uint32_t cnt = first < ntiles ? (ntiles - first < per ? ntiles - first : per) : 0u;
      if (local >= cnt) break;
      tt = first + (rev ? cnt - 1u - local : local);
    } else {
      tt = blockIdx.x + it * G;
      if (tt >= ntiles) break;
      if (rev) tt = ntiles - 1u - tt;
    }
    uint32_t dom, start, count;
    if (tiles != nullptr) {
      const Tile tl = tiles[tt];
      dom = tl.dom;
      start = tl.start;
      count = tl.count;
    } else {
      dom = 0;
      start = tt * tile_nodes;
      const uint32_t N = doms[0].N;
      count = (N - start < tile_nodes) ? N - start : tile_nodes;
    }
    const DomainDev& Dm = doms[dom];
    const Coef<T>& C = coef<T>(Dm);
    gmem<S>* fa = to_global((S*)Dm.fa);
    gmem<S>* fb = to_global((S*)Dm.fb);
    gmem<S>* fin;
    gmem<S>* fout;
    if constexpr (PH == PH_AB) {
      fin = parity ? fb : fa;
      fout = parity ? fa : fb;
    } else {
      fin = fa;
      fout = fa;
    }
    using NSp = NodeStep<L, ST, EQ, FORCE, BC, PH, BUF>;
    const auto rin = StreamRes<BUF>::template make<Lat<L>::Q>(fin, BUF ? Dm.ld : 0u);
    const auto rout = StreamRes<BUF>::template make<Lat<L>::Q>((const gmem<S>*)fout, BUF ? Dm.ld : 0u);
    if constexpr (NPT == 2) {
      for (uint32_t i = threadIdx.x; i < count; i += 2 * blockDim.x) {
        const uint32_t i1 = i + blockDim.x;
        NSp a, b;
        a.load(Dm, C, fin, rin, start + i, true);
        b.load(Dm, C, fin, rin, start + (i1 < count ? i1 : i), i1 < count);
        a.finish(Dm, C, fout, rout);
        b.finish(Dm, C, fout, rout);
      }
    } else {
      for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) {
        NSp a;
        a.load(Dm, C, fin, rin, start + i, true);
        a.finish(Dm, C, fout, rout);
      }
    }
  }
}

// One step of a single domain fused with its local outputs (stress / strain
// rate or grad phi of the state the step starts from, computed from the loaded
// deviations in the step's working precision).  One workgroup per tile, one
// node per thread, 64-bit addressing.
template <int L, int ST, int EQ, int FORCE, int BC, int PH>
__global__ void __launch_bounds__(256)
    k_step_local(const DomainDev* __restrict__ doms, uint32_t tile_nodes, uint32_t parity, void* out, int kind,
                 int out_f32, int alternate) {
  using SS = Store<ST>;
  using S = typename SS::S;
  using T = typename SS::T;
  const DomainDev& Dm = doms[0];
  const Coef<T>& C = coef<T>(Dm);
  const uint32_t tile = (alternate && (parity & 1u)) ? gridDim.x - 1u - blockIdx.x : blockIdx.x;
  const uint32_t N = Dm.N, start = tile * tile_nodes;
  if (start >= N) return;
  const uint32_t count = (N - start < tile_nodes) ? N - start : tile_nodes;
  gmem<S>* fa = to_global((S*)Dm.fa);
  gmem<S>* fb = to_global((S*)Dm.fb);
  gmem<S>* fin = (PH == PH_AB && parity) ? fb : fa;
  gmem<S>* fout = (PH == PH_AB) ? (parity ? fa : fb) : fa;
  using NSp = NodeStep<L, ST, EQ, FORCE, BC, PH, false>;
  for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) {
    NSp a;
    a.load(Dm, C, fin, 0, start + i, true);
    a.local_out(Dm, C, out, kind, out_f32);
    a.finish(Dm, C, fout, 0);
  }
}

// ----------------------------------------------------------------------------
// Decoding helpers for the companion kernels (FP64)
// ----------------------------------------------------------------------------
template <int ST, int J>
__device__ __forceinline__ double dec64(typename Store<ST>::S v, const Coef<double>& C) {
  if constexpr (ST == ST_F16)
    return (double)(float)v * C.w[J];
  else
    return (double)v;
}
template <int ST, int J>
__device__ __forceinline__ typename Store<ST>::S enc64(double v, const Coef<double>& C) {
  using S = typename Store<ST>::S;
  if constexpr (ST == ST_F16)
    return (S)(float)(v * C.iw[J]);
  else
    return (S)v;
}

// current population buffer of a domain after `parity` steps
template <int ST>
__device__ __forceinline__ typename Store<ST>::S* current_buffer(const DomainDev& Dm, uint32_t parity,
                                                                 bool ab) {
  using S = typename Store<ST>::S;
  return (ab && parity) ? (S*)Dm.fb : (S*)Dm.fa;
}

// Gather the deviations d_j of node idx (paper order, FP64).
template <int L, int ST, int BC, bool SWAPPED>
__device__ __forceinline__ void gather64(const DomainDev& Dm, const typename Store<ST>::S* f,
                                         uint32_t idx, double (&d)[Lat<L>::Q]) {
  constexpr int D = Lat<L>::D;
  Geo<D> g;
  if constexpr (SWAPPED) g.make(Dm, idx);
  static_for<0, Lat<L>::Q>([&](auto j_) {
    constexpr int J = decltype(j_)::value;
    d[J] = dec64<ST, J>(f[read_elem<L, BC, SWAPPED, J>(Dm, g, idx)], Dm.cd);
  });
}

// rho' = sum d_j and the first moment sum c_j d_j of node idx
template <int L>
__device__ __forceinline__ void first_moments(const DomainDev& Dm, const double (&d)[Lat<L>::Q],
                                              double& drho, double (&m1)[3]) {
  drho = 0.0;
  m1[0] = m1[1] = m1[2] = 0.0;
  static_for<0, Lat<L>::Q>([&](auto j_) {
    constexpr int J = decltype(j_)::value;
    drho += d[J];
    if constexpr (Lat<L>::e(J, 0) != 0) m1[0] += (double)Lat<L>::e(J, 0) * d[J];
    if constexpr (Lat<L>::e(J, 1) != 0) m1[1] += (double)Lat<L>::e(J, 1) * d[J];
    if constexpr (Lat<L>::e(J, 2) != 0) m1[2] += (double)Lat<L>::e(J, 2) * d[J];
  });
  m1[0] *= Dm.cd.c[0];
  m1[1] *= Dm.cd.c[1];
  m1[2] *= Dm.cd.c[2];
}

// Half-step source corrections of node idx in FP64 (eq. 2-4): dt S / 2 (0 in
// the gamma = 0 form and at the diffusive scaling), dt F / 2 and dt cs2 S / 2,
// from the parameter set or, when fields are attached, from the node's values.
struct HalfSrc {
  double source, force[3], cs2_source;
};
__device__ __forceinline__ HalfSrc half_sources(const DomainDev& Dm, uint32_t idx) {
  const Coef<double>& C = Dm.cd;
  HalfSrc h;
  if (!Dm.src_field) {
    h.source = C.half_source;
    for (int a = 0; a < 3; ++a) h.force[a] = C.half_force[a];
    h.cs2_source = C.half_cs2_source;
    return h;
  }
  const bool dbl = Dm.storage == ST_F64;
  auto at = [&](const void* p, size_t i) {
    return dbl ? ((const double*)p)[i] : (double)((const float*)p)[i];
  };
  const double S = Dm.src ? at(Dm.src, idx) : 0.0;
  h.source = C.half_src_factor * S;
  h.cs2_source = C.half_dt_cs2 * S;
  const int d = (Dm.lattice == LAT_Q9 || Dm.lattice == LAT_Q5) ? 2 : 3;
  for (int a = 0; a < 3; ++a)
    h.force[a] = (Dm.frc && Dm.equation == EQ_NSE && a < d) ? C.half_dt * at(Dm.frc, (size_t)a * Dm.N + idx) : 0.0;
  return h;
}

// rho (or phi) and u of node idx (eq. 2-4-1 / eq. 2-4-2)
template <int L, int ST, int EQ, int BC, bool SWAPPED>
__device__ __forceinline__ void macro_node(const DomainDev& Dm, const typename Store<ST>::S* f,
                                           uint32_t idx, double& rho, double (&u)[3],
                                           double& drho_out) {
  double d[Lat<L>::Q];
  gather64<L, ST, BC, SWAPPED>(Dm, f, idx, d);
  double drho, m1[3];
  first_moments<L>(Dm, d, drho, m1);
  const Coef<double>& C = Dm.cd;
  const HalfSrc h = half_sources(Dm, idx);
  rho = C.rho0 + drho + h.source;
  drho_out = drho + h.source;
  if constexpr (EQ == EQ_NSE) {
    const double ir = 1.0 / (C.hl ? C.rho0 : rho);   // He-Luo: rho0 u = j
    u[0] = (m1[0] + h.force[0]) * ir;
    u[1] = (m1[1] + h.force[1]) * ir;
    u[2] = (m1[2] + h.force[2]) * ir;
  } else {
    u[0] = C.adv[0];
    u[1] = C.adv[1];
    u[2] = C.adv[2];
  }
}

template <int L, int ST, int EQ, int BC, bool SWAPPED>
__global__ void __launch_bounds__(256)
    k_moments(const DomainDev* __restrict__ doms, uint32_t dom, uint32_t parity, int ab, void* rho_out,
              void* u_out, int out_f32) {
  const DomainDev& Dm = doms[dom];
  const auto* f = current_buffer<ST>(Dm, parity, ab);
  constexpr int D = Lat<L>::D;
  const uint32_t N = Dm.N;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
    double rho, u[3], drho;
    if (BC == 1 && Dm.has_solid && Dm.solid[idx]) {
      rho = Dm.cd.rho0;
      u[0] = u[1] = u[2] = 0.0;
    } else {
      macro_node<L, ST, EQ, BC, SWAPPED>(Dm, f, idx, rho, u, drho);
    }
    if (out_f32) {
      ((float*)rho_out)[idx] = (float)rho;
      if (u_out)
        for (int a = 0; a < D; ++a) ((float*)u_out)[(size_t)a * N + idx] = (float)u[a];
    } else {
      ((double*)rho_out)[idx] = rho;
      if (u_out)
        for (int a = 0; a < D; ++a) ((double*)u_out)[(size_t)a * N + idx] = u[a];
    }
  }
}

template <int L, int ST, int BC, bool SWAPPED>
__global__ void __launch_bounds__(256)
    k_populations(const DomainDev* __restrict__ doms, uint32_t dom, uint32_t parity, int ab,
                  double* out) {
  const DomainDev& Dm = doms[dom];
  const auto* f = current_buffer<ST>(Dm, parity, ab);
  const uint32_t N = Dm.N;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
    if (BC == 1 && Dm.has_solid && Dm.solid[idx]) {
      for (int j = 0; j < Lat<L>::Q; ++j) out[(size_t)j * N + idx] = 0.0;
      continue;
    }
    double d[Lat<L>::Q];
    gather64<L, ST, BC, SWAPPED>(Dm, f, idx, d);
    static_for<0, Lat<L>::Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      out[(size_t)J * N + idx] = Dm.cd.w[J] * Dm.cd.rho0 + d[J];
    });
  }
}

// ----------------------------------------------------------------------------
// Local derivative outputs (no finite differences), FP64:
//   NSE : tau = -(I - S_2/2) [m_2^ne + dt/2 (u F + F u + (cs2 I - u u) S)]
//         (eq. 4-32-0), and the strain rate E from eq. 4-28 with
//         K_mu = rho nu I, K_mu_b = rho nu_b I (eq. 4-31):
//         tr E = tr tau / (d rho nu_b), E = (tau - (rho nu_b - 2 rho nu / d) tr E I) / (2 rho nu)
//   NCDE: -D(phi) grad phi = (1 - s1/2) (m_1^ne + dt/2 X) (eq. 4-13), X = u S, or
//         u (phi - phi_prev) / dt on rD2Q5 / rD3Q7 (eq. 4-16)
// m^ne are moments of f - f_eq with f = fbar + dt F / 2; the second moment of
// F and the first moment of the NCDE F vanish, so they are moments of fbar.
// Output component k of node i at out[k N + i]: (xx, yy, [zz,] xy, [xz, yz])
// for tau / E, (x, y[, z]) for grad phi; zero at solid nodes.
// ----------------------------------------------------------------------------

template <int L, int ST, int EQ, int BC, bool SWAPPED>
__global__ void __launch_bounds__(256)
    k_local(const DomainDev* __restrict__ doms, uint32_t dom, uint32_t parity, int ab, void* out, int kind,
            int out_f32) {
  const DomainDev& Dm = doms[dom];
  const Coef<double>& C = Dm.cd;
  const auto* f = current_buffer<ST>(Dm, parity, ab);
  constexpr int D = Lat<L>::D;
  constexpr int NC = (EQ == EQ_NSE) ? D * (D + 1) / 2 : D;
  const uint32_t N = Dm.N;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
    double res[6] = {0, 0, 0, 0, 0, 0};
    if (!(BC == 1 && Dm.has_solid && Dm.solid[idx])) {
      double d[Lat<L>::Q];
      gather64<L, ST, BC, SWAPPED>(Dm, f, idx, d);
      double prev = 0.0;
      if (Dm.hist)   // C = 0 form
        prev = (ST == ST_F64) ? ((const double*)Dm.hist)[idx] : (double)((const float*)Dm.hist)[idx];
      local_node<L, EQ, double>(Dm, C, d, prev, kind, res);
    }
    for (int k = 0; k < NC; ++k) {
      if (out_f32)
        ((float*)out)[(size_t)k * N + idx] = (float)res[k];
      else
        ((double*)out)[(size_t)k * N + idx] = res[k];
    }
  }
}

// ---- block reduction of K doubles ----
template <int K>
__device__ __forceinline__ void block_reduce_store(double (&v)[K], double* out) {
  __shared__ double sh[K][8];
  for (int k = 0; k < K; ++k) {
    double x = v[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[k] = x;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < K; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[k][w];
      out[(size_t)blockIdx.x * K + k] = s;
    }
  }
}

// partial sums per workgroup: [sum rho', sum j_x, j_y, j_z, fluid node count]
template <int L, int ST, int EQ, int BC, bool SWAPPED>
__global__ void __launch_bounds__(256)
    k_reduce(const DomainDev* __restrict__ doms, uint32_t dom, uint32_t parity, int ab,
             double* partials) {
  const DomainDev& Dm = doms[dom];
  const auto* f = current_buffer<ST>(Dm, parity, ab);
  const uint32_t N = Dm.N;
  double acc[5] = {0, 0, 0, 0, 0};
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
    if (BC == 1 && Dm.has_solid && Dm.solid[idx]) continue;
    double d[Lat<L>::Q];
    gather64<L, ST, BC, SWAPPED>(Dm, f, idx, d);
    double drho, m1[3];
    first_moments<L>(Dm, d, drho, m1);
    const HalfSrc h = half_sources(Dm, idx);
    acc[0] += drho + h.source;
    if constexpr (EQ == EQ_NSE) {
      acc[1] += m1[0] + h.force[0];
      acc[2] += m1[1] + h.force[1];
      acc[3] += m1[2] + h.force[2];
    }
    acc[4] += 1.0;
  }
  block_reduce_store<5>(acc, partials);
}

// steady residual partials: [sum |u - u_prev|^2, sum |u|^2]; stores u into prev
// (NCDE: phi instead of u)
template <int L, int ST, int EQ, int BC, bool SWAPPED>
__global__ void __launch_bounds__(256)
    k_residual(const DomainDev* __restrict__ doms, uint32_t dom, uint32_t parity, int ab, double* prev,
               int have_prev, double* partials) {
  const DomainDev& Dm = doms[dom];
  const auto* f = current_buffer<ST>(Dm, parity, ab);
  const uint32_t N = Dm.N;
  constexpr int K = (EQ == EQ_NSE) ? Lat<L>::D : 1;
  double acc[2] = {0, 0};
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
    if (BC == 1 && Dm.has_solid && Dm.solid[idx]) continue;
    double rho, u[3], drho;
    macro_node<L, ST, EQ, BC, SWAPPED>(Dm, f, idx, rho, u, drho);
    double v[3] = {u[0], u[1], u[2]};
    if constexpr (EQ != EQ_NSE) v[0] = rho;
    for (int a = 0; a < K; ++a) {
      const double old = prev[(size_t)a * N + idx];
      if (have_prev) acc[0] += (v[a] - old) * (v[a] - old);
      acc[1] += v[a] * v[a];
      prev[(size_t)a * N + idx] = v[a];
    }
  }
  block_reduce_store<2>(acc, partials);
}

// Sum of nb x K partials in a fixed order (deterministic); the result is
// valid in thread 0 of a single 256-thread workgroup.
template <int K>
__device__ __forceinline__ void sum_partials(const double* __restrict__ partials, uint32_t nb, double (&res)[K]) {
  __shared__ double sh[K][256];
  double v[K];
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
    for (int k = 0; k < K; ++k) v[k] += partials[(size_t)b * K + k];
  for (int k = 0; k < K; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (uint32_t t = 0; t < blockDim.x; ++t) s += sh[k][t];
      res[k] = s;
    }
  }
}

template <int K>
__global__ void k_reduce_final(const double* __restrict__ partials, uint32_t nb, double* out) {
  double res[K];
  sum_partials<K>(partials, nb, res);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) out[k] = res[k];
}


// ----------------------------------------------------------------------------
// Initialisation: fbar = g_eq(A, B, M) in velocity space (eq. 3-3) with
//   NSE : A = rho - rho0 - Sbar/2, B = rho u - Fbar/2,
//         M = rho u u + cs2 Sbar I / 2 [+ m_2^ne of eq. 4-34]
//   NCDE: A = phi - phi0 - S/2,    B = phi adv,  M = phi adv adv
//         (M = 0 on rD2Q5 / rD3Q7, which also set their history field to phi)
// written in the natural layout, or through the swapped addressing when the
// state is expected after an odd number of AA steps.
// ----------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void velocity_gradient(const DomainDev& Dm, const double* u, uint32_t idx,
                                                  const Geo<D>& g, double (&G)[3][3]) {
  const uint32_t N = Dm.N;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) G[a][b] = 0.0;
  for (int b = 0; b < D; ++b) {
    const int32_t op = (b == 0) ? g.ox[2] : (b == 1 ? g.oy[2] : g.oz[2]);
    const int32_t om = (b == 0) ? g.ox[0] : (b == 1 ? g.oy[0] : g.oz[0]);
    const uint32_t ip = checked_node(Dm, idx + (uint32_t)op, idx), im = checked_node(Dm, idx + (uint32_t)om, idx);
    bool okp = !g.hi[b], okm = !g.lo[b];
    if (Dm.has_solid) {
      okp = okp && !Dm.solid[ip];
      okm = okm && !Dm.solid[im];
    }
    const double h = Dm.cd.c[b] * Dm.cd.dt;
    for (int a = 0; a < D; ++a) {
      const double* ua = u + (size_t)a * N;
      if (okp && okm)
        G[a][b] = (ua[ip] - ua[im]) / (2.0 * h);
      else if (okp)
        G[a][b] = (ua[ip] - ua[idx]) / h;
      else if (okm)
        G[a][b] = (ua[idx] - ua[im]) / h;
    }
  }
}

template <int L, int ST, int EQ, bool SWAPPED>
__global__ void __launch_bounds__(256)
    k_init(const DomainDev* __restrict__ doms, uint32_t dom, uint32_t parity, int ab,
           const double* __restrict__ rho_in, const double* __restrict__ u_in, int with_fne) {
  using S = typename Store<ST>::S;
  constexpr int D = Lat<L>::D;
  const DomainDev& Dm = doms[dom];
  const Coef<double>& C = Dm.cd;
  S* f = current_buffer<ST>(Dm, parity, ab);
  const uint32_t N = Dm.N;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
    Geo<D> g;
    g.make(Dm, idx);
    const double r = rho_in ? rho_in[idx] : C.rho0;
    double A, B[3] = {0, 0, 0}, M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const HalfSrc h = half_sources(Dm, idx);
    if constexpr (EQ == EQ_NSE) {
      double u[3] = {0, 0, 0};
      if (u_in)
        for (int a = 0; a < D; ++a) u[a] = u_in[(size_t)a * N + idx];
      const double ru = C.hl ? C.rho0 : r;   // He-Luo: g_eq(rho, rho0 u, rho0 u u)
      A = r - C.rho0 - h.source;
      for (int a = 0; a < 3; ++a) B[a] = ru * u[a] - h.force[a];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] = ru * u[a] * u[b] + (a == b ? h.cs2_source : 0.0);
      if (with_fne && u_in && !(Dm.has_solid && Dm.solid[idx])) {
        // m_2^ne = -(I - S2/2)^-1 tau - dt/2 (u F + F u + cs2 Sbar I)   (eq. 4-34)
        double G[3][3];
        velocity_gradient<D>(Dm, u_in, idx, g, G);
        double div = 0.0;
        for (int a = 0; a < D; ++a) div += G[a][a];
        // eq. 4-28 with the viscosity tensors of eq. 4-29
        double tau[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int a = 0; a < D; ++a)
          tau[a][a] = ru * (Dm.ic.nu_diag[a] * (2.0 * G[a][a] - 2.0 / D * div) + Dm.ic.nu_b_ax[a] * div);
        tau[0][1] = tau[1][0] = ru * Dm.ic.nu_pair[0] * (G[0][1] + G[1][0]);
        tau[0][2] = tau[2][0] = ru * Dm.ic.nu_pair[1] * (G[0][2] + G[2][0]);
        tau[1][2] = tau[2][1] = ru * Dm.ic.nu_pair[2] * (G[1][2] + G[2][1]);
        double mne[3][3];
        for (int a = 0; a < 3; ++a) {
          double s = 0.0;
          for (int b = 0; b < 3; ++b) s += Dm.ic.Kd[a][b] * tau[b][b];
          mne[a][a] = -s;
        }
        mne[0][1] = mne[1][0] = -Dm.ic.k_off[0] * tau[0][1];
        mne[0][2] = mne[2][0] = -Dm.ic.k_off[1] * tau[0][2];
        mne[1][2] = mne[2][1] = -Dm.ic.k_off[2] * tau[1][2];
        // (the half-step corrections already carry the factor dt / 2)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            M[a][b] += mne[a][b] - (u[a] * h.force[b] + h.force[a] * u[b] + (a == b ? h.cs2_source : 0.0));
      }
    } else {
      A = r - C.rho0 - h.source;
      for (int a = 0; a < 3; ++a) B[a] = r * C.adv[a];
      if constexpr (!Lat<L>::linear)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) M[a][b] = r * C.adv_c[a] * C.adv_c[b];   // 0 in the C = 0 forms
      if (Dm.hist && !(Dm.has_solid && Dm.solid[idx]))
        ((typename Store<ST>::T*)Dm.hist)[idx] = (typename Store<ST>::T)r;   // dB/dt = 0 at the first step
    }
    // g_eq_j = w_j (A + c_j.B / cs2 + sum_a M_aa (c_ja^2 - cs2) / (cs2 (c_a^2 - cs2))
    //               + sum_{a<b} M_ab c_ja c_jb / cs2^2)
    const double ics2 = C.inv_cs2;
    double qa[3], qo[3];
    for (int a = 0; a < 3; ++a) qa[a] = 1.0 / (C.c[a] * C.c[a] - C.cs2);
    qo[0] = C.c[0] * C.c[1] * ics2 * ics2;
    qo[1] = C.c[0] * C.c[2] * ics2 * ics2;
    qo[2] = C.c[1] * C.c[2] * ics2 * ics2;
    static_for<0, Lat<L>::Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      constexpr int ex = Lat<L>::e(J, 0), ey = Lat<L>::e(J, 1), ez = Lat<L>::e(J, 2);
      double v = A + ics2 * (ex * C.c[0] * B[0] + ey * C.c[1] * B[1] + ez * C.c[2] * B[2]);
      const int e[3] = {ex, ey, ez};
      for (int a = 0; a < D; ++a) {
        const double cja2 = e[a] * e[a] * C.c[a] * C.c[a];
        v += M[a][a] * (cja2 - C.cs2) * ics2 * qa[a];
      }
      v += M[0][1] * (ex * ey) * qo[0];
      if constexpr (D == 3) {
        v += M[0][2] * (ex * ez) * qo[1];
        v += M[1][2] * (ey * ez) * qo[2];
      }
      v *= C.w[J];
      size_t e_out;
      if constexpr (SWAPPED) {
        // f_J(x) lives in slot opp(J) of x - e_J, or slot J of x if that link bounces
        constexpr int O = Lat<L>::opp(J);
        bool b = false;
        b = g.template bounce<L, O>(Dm, idx);
        e_out = b ? (size_t)J * Dm.ld + idx : (size_t)O * Dm.ld + g.template nbr<L, O>(Dm, idx);
      } else {
        e_out = (size_t)J * Dm.ld + idx;
      }
      if (!(Dm.has_solid && Dm.solid[idx])) f[e_out] = enc64<ST, J>(v, C);
    });
  }
}

template <int L>
__global__ void __launch_bounds__(256) k_links(const DomainDev* __restrict__ doms, uint32_t dom, void* out) {
  using LW = typename LinkBits<L>::W;
  const DomainDev& Dm = doms[dom];
  const uint32_t N = Dm.N;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
    Geo<Lat<L>::D> g;
    g.make(Dm, idx);
    LW bits = 0;
    static_for<1, Lat<L>::Q>([&](auto j_) {
      constexpr int J = decltype(j_)::value;
      if (g.template bounce<L, J>(Dm, idx)) bits |= (LW)1 << J;
    });
    if (Dm.has_solid && Dm.solid[idx]) bits |= LinkBits<L>::kSolid;
    ((LW*)out)[idx] = bits;
  }
}

// ----------------------------------------------------------------------------
// Host-side launch descriptors (defined per lattice/storage translation unit)
// ----------------------------------------------------------------------------
struct StepLaunch {
  const DomainDev* doms;
  const Tile* tiles;
  uint32_t ntiles, tile_nodes, parity, flags;
  uint32_t lds_bytes;  // dynamic LDS per workgroup: caps resident workgroups per CU
  int eq, force, bc, phase;
  unsigned grid, block;
  hipStream_t stream;
  // fused local outputs (k_step_local) when local_out is set
  void* local_out;
  int local_kind, local_f32;
};
struct AuxLaunch {
  const DomainDev* doms;
  uint32_t dom, parity;
  int ab, eq, bc, swapped;
  unsigned grid, block;
  hipStream_t stream;
  // kind-specific
  void* out0;
  void* out1;
  const double* in0;
  const double* in1;
  int flag;
  int kind;   // k_local: GRAD_*
};

template <int L, int ST>
hipError_t launch_step(const StepLaunch& a);
template <int L, int ST>
hipError_t launch_init(const AuxLaunch& a);
template <int L, int ST>
hipError_t launch_moments(const AuxLaunch& a);
template <int L, int ST>
hipError_t launch_populations(const AuxLaunch& a);
template <int L, int ST>
hipError_t launch_reduce(const AuxLaunch& a);
template <int L, int ST>
hipError_t launch_residual(const AuxLaunch& a);
template <int L, int ST>
hipError_t launch_local(const AuxLaunch& a);
template <int L>
hipError_t launch_links(const DomainDev* doms, uint32_t dom, void* out, unsigned grid, hipStream_t s);
hipError_t launch_reduce_final(const double* partials, uint32_t nb, double* out, int K, hipStream_t s);
hipError_t launch_reduce_final_mass(const double* partials, uint32_t nb, double rho0, double* out, hipStream_t s);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace rmrt
