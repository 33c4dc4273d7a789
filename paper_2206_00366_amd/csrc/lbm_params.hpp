// Parameter block shared by the host code and the kernels of this library
// (one record per domain, resident in device memory, read with scalar loads).
#pragma once

#include <stdint.h>

namespace rmrt {

enum { LAT_Q9 = 0, LAT_Q19 = 1, LAT_Q27 = 2, LAT_Q5 = 3, LAT_Q7 = 4 };
// EQ_NCDE_C0: the NCDE in the C = 0 form of eq. 4-16 on the full lattices
// (rD2Q5 / rD3Q7 always take that form under EQ_NCDE)
// EQ_NSE_BASIS: the NSE relaxed in another moment basis of eq. 5-1-1 / 5-1-2,
// the central (rD2Q9, rD3Q27), Hermite (rD2Q9, rD3Q19, rD3Q27) or
// central-Hermite one (Coef::basis)
enum { EQ_NSE = 0, EQ_NCDE = 1, EQ_NCDE_C0 = 2, EQ_NSE_BASIS = 3 };
enum : uint32_t { BASIS_CENTRAL = 1u, BASIS_HERMITE = 2u, BASIS_BHLL = 4u };
// source terms of a step: none, the parameter set's constants, or per-node
// fields (mass or NCDE source, body force; read per node and step)
enum { F_NONE = 0, F_CONST = 1, F_FIELD = 2 };
enum { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2 };
enum { PH_AB = 0, PH_AA_EVEN = 1, PH_AA_ODD = 2 };

// Coefficients in the working precision T.  Tables indexed by a tensor slot n
// (n = a + 3 b + 9 p for the raw moment c_x^a c_y^b c_z^p) are in the scaled
// basis m~ = D^-1 m of the integer factor M~.
template <typename T>
struct Coef {
  T rho0, cs2, inv_cs2, dt;
  T c[3], inv_c[3];
  T w[27], iw[27];          // weights in paper order and their reciprocals
  // the same by weight class (0 rest, 1-3 x/y/z axes, 4-6 xy/xz/yz edges, 7
  // corners): every velocity of a class has the same weight (Sec. III), so
  // the step reads 8 values instead of q
  T wc[8], iwc[8];
  // scaled raw moment n of g_eq(A, B, M):
  //   A E0[n] + B_odd E1[n] + sum_a M_aa E2[n][a] + M_pair E3[n]
  T E0[27], E1[27], E2[27][3], E3[27];
  T Sd[3][3];               // scaled second-order diagonal block: Sbar_ab c_b^2 / c_a^2
  T s_off[3];               // rates of the xy, xz, yz second moments
  T s_hi;                   // rate of the higher moments
  T IhS[3][3];              // I - Sbar/2 (unscaled), for M_2G
  T ihs_off[3];             // 1 - s_off/2
  T force[3], half_force[3];
  T source, half_source, cs2_source, half_cs2_source;
  T adv[3], D0, D2, inv_cs2_dt, inv_dt;
  T adv_c[3];               // NCDE: adv in C = phi u u (0 at the diffusive scaling, eq. 4-17)
  T adv_g[3];               // NCDE: adv in M_1G (0 at the diffusive scaling: G = 0)
  // per-node source fields: source = dt S, half_source = half_src_factor S
  // (0.5 dt, or 0 in the gamma = 0 form and at the diffusive scaling),
  // cs2_source = dt_cs2 S, half_cs2_source = half_dt_cs2 S, force = dt F,
  // half_force = half_dt F
  T half_dt, dt_cs2, half_dt_cs2, half_src_factor;
  uint32_t hl;              // He-Luo equilibrium (1) or eq. NSEfeq (0)
  uint32_t hist_g;          // NCDE: G from dB/dt with the previous step's phi (C = 0 form of eq. 4-16)
  uint32_t basis;           // EQ_NSE_BASIS: BASIS_CENTRAL | BASIS_HERMITE, or BASIS_BHLL
  T hth[3];                 // Hermite basis: cs2 / c_a^2 (H_2 = e^2 - cs2 / c_a^2 in the scaled basis)
  // BHLL basis (rD2Q9): the relaxation N^-1 Sbar_B N written in the scaled raw
  // basis, over the non-conserved tensor slots 2, 4, 5, 6, 7, 8
  T rb[6][6];
};

// Initialisation-only quantities (always FP64).
struct InitCoef {
  double Kd[3][3];   // (I - Sbar/2)^-1 on the diagonal second moments
  double k_off[3];   // 1 / (1 - s_off/2)
  double nu, nu_b;
  double nu_diag[3], nu_pair[3], nu_b_ax[3];   // viscosity tensor entries (eq. 4-29)
  // strain rate from the stress (eq. 4-28 inverted with the tensors of eq. 4-29),
  // per axis a < d: 1 / (2 nu_aa) and nu_b,a - 2 nu_aa / d; 1 / (1 + sum of
  // their products); 1 / (2 nu_ab) per pair
  double inv2nu_diag[3], bulk_excess[3], inv_trace_den, inv2nu_pair[3];
};

struct DomainDev {
  Coef<double> cd;
  Coef<float> cf;
  InitCoef ic;
  uint32_t nx, ny, nz, N;
  uint32_t ld;              // stream stride: population j of node i is element j * ld + i
  uint32_t nxny;
  uint32_t mnx, mnxny;      // floor(2^32 / divisor) (0xffffffff for divisor 1)
  uint32_t walls;           // RMRT_WALL_* bits
  uint32_t has_solid;
  uint32_t lattice, equation, storage;
  void* fa;                 // population buffer 0
  void* fb;                 // population buffer 1 (two-lattice pattern)
  const uint8_t* solid;     // 1 byte per node or null
  const void* links;        // per-node link bits (uint16 for q <= 15, uint32 otherwise) or null:
                            // bit j = link x -> x + e_j hits a wall or solid; top bit = solid node
  void* hist;               // C = 0 NCDE form: phi of the previous step per node (double for FP64
                            // storage, float otherwise); null otherwise
  // per-node source fields (working precision: double for FP64 storage, float
  // otherwise), used when src_field is set: S (N values; null = 0), F (d x N
  // SoA body force, NSE; null = 0), and in the gamma = 0 NCDE form the
  // source of the previous step (N values, library-owned; null otherwise)
  const void* src;
  const void* frc;
  void* sprev;
  uint32_t src_field;
  // checked builds (RMRT_CHECKED): the node-index bound that every neighbour
  // index is tested against (N unless a test lowers it) and the device
  // counter of indices found outside it; unused by the production build
  uint32_t oob_limit;
  uint32_t* oob;
};

// One unit of persistent-kernel work: nodes [start, start + count) of a domain.
struct Tile {
  uint32_t dom, start, count, pad;
};

}  // namespace rmrt
