// lb_blocked_f64_q9.hip -- instantiates the temporally blocked kernels (lb_blocked.h)
// for FP64 populations on D2Q9: single-grid and batched launches.
#include "lb_blocked.h"

namespace lbw {
LBW_BLOCKED_UNIT(double, 9, f64_q9)
}  // namespace lbw
