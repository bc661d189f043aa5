// lb_blocked_f32_q9.hip -- instantiates the temporally blocked kernels (lb_blocked.h)
// for FP32 populations on D2Q9: single-grid and batched launches.
#include "lb_blocked.h"

namespace lbw {
LBW_BLOCKED_UNIT(float, 9, f32_q9)
}  // namespace lbw
