// Kernel launchers replaced by stubs for the sanitizer build of the host code:
// the host-only paths it exercises (parameter derivation and validation,
// argument checks) never launch a kernel, and a stub that is reached fails.
#include "../../paper_2206_00366_amd/csrc/lbm_kernels.hpp"

namespace rmrt {

template <int L, int ST>
hipError_t launch_step(const StepLaunch&) { return hipErrorNotSupported; }
template <int L, int ST>
hipError_t launch_init(const AuxLaunch&) { return hipErrorNotSupported; }
template <int L, int ST>
hipError_t launch_moments(const AuxLaunch&) { return hipErrorNotSupported; }
template <int L, int ST>
hipError_t launch_populations(const AuxLaunch&) { return hipErrorNotSupported; }
template <int L, int ST>
hipError_t launch_reduce(const AuxLaunch&) { return hipErrorNotSupported; }
template <int L, int ST>
hipError_t launch_residual(const AuxLaunch&) { return hipErrorNotSupported; }
template <int L, int ST>
hipError_t launch_local(const AuxLaunch&) { return hipErrorNotSupported; }
template <int L>
hipError_t launch_links(const DomainDev*, uint32_t, void*, unsigned, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reduce_final(const double*, uint32_t, double*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reduce_final_mass(const double*, uint32_t, double, double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_stream_copy(void*, const void*, size_t, hipStream_t) { return hipErrorNotSupported; }

#define STUBS(L, ST)                                                   \
  template hipError_t launch_step<L, ST>(const StepLaunch&);          \
  template hipError_t launch_init<L, ST>(const AuxLaunch&);           \
  template hipError_t launch_moments<L, ST>(const AuxLaunch&);        \
  template hipError_t launch_populations<L, ST>(const AuxLaunch&);    \
  template hipError_t launch_reduce<L, ST>(const AuxLaunch&);         \
  template hipError_t launch_residual<L, ST>(const AuxLaunch&);       \
  template hipError_t launch_local<L, ST>(const AuxLaunch&);
#define STUBS_L(L) \
  STUBS(L, ST_F64) STUBS(L, ST_F32) STUBS(L, ST_F16) \
  template hipError_t launch_links<L>(const DomainDev*, uint32_t, void*, unsigned, hipStream_t);
STUBS_L(LAT_Q9)
STUBS_L(LAT_Q19)
STUBS_L(LAT_Q27)
STUBS_L(LAT_Q5)
STUBS_L(LAT_Q7)

}  // namespace rmrt
