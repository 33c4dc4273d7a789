// Kernel instances for LAT_Q5 with ST_F64 storage.
#include "lbm_launch.hpp"
namespace rmrt {
RMRT_INSTANTIATE(LAT_Q5, ST_F64)
RMRT_INSTANTIATE_LINKS(LAT_Q5)
}  // namespace rmrt
