// lb_blocked_f16_q5.hip -- instantiates the temporally blocked kernels (lb_blocked.h)
// for FP16-stored populations on D2Q5: single-grid and batched launches.
#include "lb_blocked.h"

namespace lbw {
LBW_BLOCKED_UNIT(_Float16, 5, f16_q5)
}  // namespace lbw
