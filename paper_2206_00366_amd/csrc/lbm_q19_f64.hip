// Kernel instances for LAT_Q19 with ST_F64 storage.
#include "lbm_launch.hpp"
namespace rmrt {
RMRT_INSTANTIATE(LAT_Q19, ST_F64)
RMRT_INSTANTIATE_LINKS(LAT_Q19)
}  // namespace rmrt
