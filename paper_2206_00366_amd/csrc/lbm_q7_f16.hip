// Kernel instances for LAT_Q7 with ST_F16 storage.
#include "lbm_launch.hpp"
namespace rmrt {
RMRT_INSTANTIATE(LAT_Q7, ST_F16)
}  // namespace rmrt
