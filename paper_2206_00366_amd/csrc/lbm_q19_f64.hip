// Kernel instances for LAT_Q19 with ST_F64 storage.
#include "lbm_launch.hpp"
namespace rmrt {
RMRT_INSTANTIATE(LAT_Q19, ST_F64)
}  // namespace rmrt
