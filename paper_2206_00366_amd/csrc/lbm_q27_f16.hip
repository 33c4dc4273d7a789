// Kernel instances for LAT_Q27 with ST_F16 storage.
#include "lbm_launch.hpp"
namespace rmrt {
RMRT_INSTANTIATE(LAT_Q27, ST_F16)
}  // namespace rmrt
