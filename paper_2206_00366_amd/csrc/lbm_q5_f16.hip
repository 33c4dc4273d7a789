// Kernel instances for LAT_Q5 with ST_F16 storage.
#include "lbm_launch.hpp"
namespace rmrt {
RMRT_INSTANTIATE(LAT_Q5, ST_F16)
}  // namespace rmrt
