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

// The mass and momentum of k_reduce's partials [sum rho', sum j, fluid count]:
// out = [count rho0 + sum rho', sum j_x, sum j_y, sum j_z], the values the host
// forms from k_reduce_final's sums (the product and the sum rounded separately).
__global__ void k_reduce_final_mass(const double* __restrict__ partials, uint32_t nb, double rho0, double* out) {
  double res[5];
  sum_partials<5>(partials, nb, res);
  if (threadIdx.x == 0) {
#pragma clang fp contract(off)
    out[0] = res[4] * rho0 + res[0];
    out[1] = res[1];
    out[2] = res[2];
    out[3] = res[3];
  }
}

hipError_t launch_reduce_final_mass(const double* partials, uint32_t nb, double rho0, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final_mass, dim3(1), dim3(256), 0, s, partials, nb, rho0, out);
  return hipGetLastError();
}

}  // namespace rmrt

namespace rmrt {

// HBM ceiling probe: one 16-byte vector per thread, one pass (no grid-stride
// loop); measured on MI355X this is the fastest plain copy shape.
__global__ void __launch_bounds__(256) k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     size_t n16) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  const size_t blocks = (n16 + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

}  // namespace rmrt
