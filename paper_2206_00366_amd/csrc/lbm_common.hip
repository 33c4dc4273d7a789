// Lattice-independent kernels.
#include "lbm_kernels.hpp"

namespace rmrt {

hipError_t launch_reduce_final(const double* partials, uint32_t nb, double* out, int K, hipStream_t s) {
  if (K == 5)
    hipLaunchKernelGGL((k_reduce_final<5>), dim3(1), dim3(256), 0, s, partials, nb, out);
  else
    hipLaunchKernelGGL((k_reduce_final<2>), dim3(1), dim3(256), 0, s, partials, nb, out);
  return hipGetLastError();
}

}  // namespace rmrt
