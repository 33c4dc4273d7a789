// Kernel instances for LAT_Q9 with ST_F32 storage.
#include "lbm_launch.hpp"
namespace rmrt {
RMRT_INSTANTIATE(LAT_Q9, ST_F32)
}  // namespace rmrt
