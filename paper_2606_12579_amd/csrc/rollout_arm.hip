// Arm-agent instantiations of the rollout kernel (serial chains moved through
// their joints, any heuristic), compiled apart to keep builds parallel.
#include "rollout_kernel.h"

namespace gm {

KFn pick_kernel_arm(int AW, int W, bool wg, int cut)
{
    return pick_kernel_t<true, 2>(AW, W, wg, cut, false);
}

}  // namespace gm
