// Host launchers: map runtime enumerations onto kernel template instances.
#pragma once

#include "lbm_kernels.hpp"

namespace rmrt {

// Field sources, the C = 0 NCDE form and the basis collisions (central,
// Hermite, BHLL) have a one-node-per-thread kernel only: with STEP_WIDE_TILES
// it walks each 512-node tile in two passes.
template <int L, int ST, int EQ, int F, int BC, int PH, bool BUF>
void do_step_npt(const StepLaunch& a) {
  if constexpr (F == F_FIELD || EQ == EQ_NCDE_C0 || EQ == EQ_NSE_BASIS)
    hipLaunchKernelGGL((k_step<L, ST, EQ, F, BC, PH, 1, BUF>), dim3(a.grid), dim3(a.block), a.lds_bytes, a.stream,
                       a.doms, a.tiles, a.ntiles, a.tile_nodes, a.parity, a.flags);
  else if (a.flags & STEP_WIDE_TILES)
    hipLaunchKernelGGL((k_step<L, ST, EQ, F, BC, PH, 2, BUF>), dim3(a.grid), dim3(a.block), a.lds_bytes, a.stream,
                       a.doms, a.tiles, a.ntiles, a.tile_nodes, a.parity, a.flags);
  else
    hipLaunchKernelGGL((k_step<L, ST, EQ, F, BC, PH, 1, BUF>), dim3(a.grid), dim3(a.block), a.lds_bytes, a.stream,
                       a.doms, a.tiles, a.ntiles, a.tile_nodes, a.parity, a.flags);
}
// STEP_BUFFER_OFFSETS reaches here only for buffers below 4 GiB (the host
// clears it otherwise).
template <int L, int ST, int EQ, int F, int BC, int PH>
hipError_t do_step(const StepLaunch& a) {
  if (a.local_out) {
    if constexpr (F == F_FIELD || EQ == EQ_NSE_BASIS) {
      return hipErrorInvalidValue;   // local outputs: raw-moment model, constant sources (host-checked)
    } else {
      hipLaunchKernelGGL((k_step_local<L, ST, EQ, F, BC, PH>), dim3(a.ntiles), dim3(a.block), a.lds_bytes,
                         a.stream, a.doms, a.tile_nodes, a.parity, a.local_out, a.local_kind, a.local_f32,
                         (int)((a.flags & STEP_ALTERNATE_ORDER) != 0));
      return hipGetLastError();
    }
  }
  if (a.flags & STEP_BUFFER_OFFSETS)
    do_step_npt<L, ST, EQ, F, BC, PH, true>(a);
  else
    do_step_npt<L, ST, EQ, F, BC, PH, false>(a);
  return hipGetLastError();
}
template <int L, int ST, int EQ, int F, int BC>
hipError_t step_ph(const StepLaunch& a) {
  switch (a.phase) {
    case PH_AB: return do_step<L, ST, EQ, F, BC, PH_AB>(a);
    case PH_AA_EVEN: return do_step<L, ST, EQ, F, BC, PH_AA_EVEN>(a);
    case PH_AA_ODD: return do_step<L, ST, EQ, F, BC, PH_AA_ODD>(a);
  }
  return hipErrorInvalidValue;
}
template <int L, int ST, int EQ, int F>
hipError_t step_bc(const StepLaunch& a) {
  switch (a.bc) {
    case 0: return step_ph<L, ST, EQ, F, 0>(a);
    case 1: return step_ph<L, ST, EQ, F, 1>(a);
    case 2: return step_ph<L, ST, EQ, F, 2>(a);
  }
  return hipErrorInvalidValue;
}
template <int L, int ST, int EQ>
hipError_t step_f(const StepLaunch& a) {
  switch (a.force) {
    case F_NONE: return step_bc<L, ST, EQ, F_NONE>(a);
    case F_CONST: return step_bc<L, ST, EQ, F_CONST>(a);
    case F_FIELD: return step_bc<L, ST, EQ, F_FIELD>(a);
  }
  return hipErrorInvalidValue;
}
template <int L, int ST>
hipError_t launch_step(const StepLaunch& a) {
  if constexpr (Lat<L>::linear) {   // rD2Q5 / rD3Q7 carry the NCDE only, always in the C = 0 form
    return (a.eq == EQ_NCDE || a.eq == EQ_NCDE_C0) ? step_f<L, ST, EQ_NCDE>(a) : hipErrorInvalidValue;
  } else {
    switch (a.eq) {
      case EQ_NSE: return step_f<L, ST, EQ_NSE>(a);
      case EQ_NCDE: return step_f<L, ST, EQ_NCDE>(a);
      case EQ_NCDE_C0: return step_f<L, ST, EQ_NCDE_C0>(a);
      case EQ_NSE_BASIS: return step_f<L, ST, EQ_NSE_BASIS>(a);
    }
    return hipErrorInvalidValue;
  }
}

// ---- companions: dispatch over (eq, bc, swapped) ----
#define RMRT_AUX_DISPATCH(KCALL)                                       \
  if (a.eq == EQ_NSE) {                                                \
    if (a.bc) {                                                        \
      if (a.swapped) { KCALL(EQ_NSE, 1, true); } else { KCALL(EQ_NSE, 1, false); } \
    } else {                                                           \
      if (a.swapped) { KCALL(EQ_NSE, 0, true); } else { KCALL(EQ_NSE, 0, false); } \
    }                                                                  \
  } else {                                                             \
    if (a.bc) {                                                        \
      if (a.swapped) { KCALL(EQ_NCDE, 1, true); } else { KCALL(EQ_NCDE, 1, false); } \
    } else {                                                           \
      if (a.swapped) { KCALL(EQ_NCDE, 0, true); } else { KCALL(EQ_NCDE, 0, false); } \
    }                                                                  \
  }                                                                    \
  return hipGetLastError();

template <int L, int ST>
hipError_t launch_moments(const AuxLaunch& a) {
#define K_MOM(EQ, BC, SW)                                                                          \
  hipLaunchKernelGGL((k_moments<L, ST, EQ, BC, SW>), dim3(a.grid), dim3(a.block), 0, a.stream, a.doms, \
                     a.dom, a.parity, a.ab, a.out0, a.out1, a.flag)
  RMRT_AUX_DISPATCH(K_MOM)
#undef K_MOM
}

template <int L, int ST>
hipError_t launch_reduce(const AuxLaunch& a) {
#define K_RED(EQ, BC, SW)                                                                         \
  hipLaunchKernelGGL((k_reduce<L, ST, EQ, BC, SW>), dim3(a.grid), dim3(a.block), 0, a.stream, a.doms, \
                     a.dom, a.parity, a.ab, (double*)a.out0)
  RMRT_AUX_DISPATCH(K_RED)
#undef K_RED
}

template <int L, int ST>
hipError_t launch_residual(const AuxLaunch& a) {
#define K_RES(EQ, BC, SW)                                                                           \
  hipLaunchKernelGGL((k_residual<L, ST, EQ, BC, SW>), dim3(a.grid), dim3(a.block), 0, a.stream, a.doms, \
                     a.dom, a.parity, a.ab, (double*)a.out1, a.flag, (double*)a.out0)
  RMRT_AUX_DISPATCH(K_RES)
#undef K_RES
}

template <int L, int ST>
hipError_t launch_populations(const AuxLaunch& a) {
  if (a.bc) {
    if (a.swapped)
      hipLaunchKernelGGL((k_populations<L, ST, 1, true>), dim3(a.grid), dim3(a.block), 0, a.stream,
                         a.doms, a.dom, a.parity, a.ab, (double*)a.out0);
    else
      hipLaunchKernelGGL((k_populations<L, ST, 1, false>), dim3(a.grid), dim3(a.block), 0, a.stream,
                         a.doms, a.dom, a.parity, a.ab, (double*)a.out0);
  } else {
    if (a.swapped)
      hipLaunchKernelGGL((k_populations<L, ST, 0, true>), dim3(a.grid), dim3(a.block), 0, a.stream,
                         a.doms, a.dom, a.parity, a.ab, (double*)a.out0);
    else
      hipLaunchKernelGGL((k_populations<L, ST, 0, false>), dim3(a.grid), dim3(a.block), 0, a.stream,
                         a.doms, a.dom, a.parity, a.ab, (double*)a.out0);
  }
  return hipGetLastError();
}

template <int L, int ST>
hipError_t launch_init(const AuxLaunch& a) {
#define K_INIT(EQ, SW)                                                                          \
  hipLaunchKernelGGL((k_init<L, ST, EQ, SW>), dim3(a.grid), dim3(a.block), 0, a.stream, a.doms, \
                     a.dom, a.parity, a.ab, a.in0, a.in1, a.flag)
  if (a.eq == EQ_NSE) {
    if (a.swapped) { K_INIT(EQ_NSE, true); } else { K_INIT(EQ_NSE, false); }
  } else {
    if (a.swapped) { K_INIT(EQ_NCDE, true); } else { K_INIT(EQ_NCDE, false); }
  }
#undef K_INIT
  return hipGetLastError();
}

template <int L, int ST>
hipError_t launch_local(const AuxLaunch& a) {
#define K_LOC(EQ, BC, SW)                                                                         \
  hipLaunchKernelGGL((k_local<L, ST, EQ, BC, SW>), dim3(a.grid), dim3(a.block), 0, a.stream, a.doms, \
                     a.dom, a.parity, a.ab, a.out0, a.kind, a.flag)
  RMRT_AUX_DISPATCH(K_LOC)
#undef K_LOC
}

template <int L>
hipError_t launch_links(const DomainDev* doms, uint32_t dom, void* out, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((k_links<L>), dim3(grid), dim3(256), 0, s, doms, dom, out);
  return hipGetLastError();
}

#define RMRT_INSTANTIATE_LINKS(L) template hipError_t launch_links<L>(const DomainDev*, uint32_t, void*, unsigned, hipStream_t);

#define RMRT_INSTANTIATE(L, ST)                                 \
  template hipError_t launch_step<L, ST>(const StepLaunch&);    \
  template hipError_t launch_init<L, ST>(const AuxLaunch&);     \
  template hipError_t launch_moments<L, ST>(const AuxLaunch&);  \
  template hipError_t launch_populations<L, ST>(const AuxLaunch&); \
  template hipError_t launch_reduce<L, ST>(const AuxLaunch&);   \
  template hipError_t launch_residual<L, ST>(const AuxLaunch&); \
  template hipError_t launch_local<L, ST>(const AuxLaunch&);

}  // namespace rmrt
