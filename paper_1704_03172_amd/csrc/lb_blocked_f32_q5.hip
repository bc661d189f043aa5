// lb_blocked_f32_q5.hip -- instantiates the temporally blocked kernels (lb_blocked.h)
// for FP32 populations on D2Q5: single-grid and batched launches.
#include "lb_blocked.h"

namespace lbw {
LBW_BLOCKED_UNIT(float, 5, f32_q5)
}  // namespace lbw
