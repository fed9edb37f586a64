// 6-D pose-agent instantiations of the rollout kernel (rotor and translation in
// Spin(3) x| R^3, any heuristic), compiled apart to keep builds parallel.
#include "rollout_kernel.h"

namespace gm {

KFn pick_kernel_pose(int AW, int W, bool wg, int cut)
{
    return pick_kernel_t<true, 1>(AW, W, wg, cut, false);
}

}  // namespace gm
