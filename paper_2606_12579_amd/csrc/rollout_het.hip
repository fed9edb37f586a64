// Heterogeneous-field instantiations of the rollout kernel (each agent takes the
// rotation-vector circular field, the velocity-current field or the APF from its
// heuristic code), compiled apart from the homogeneous ones to keep builds parallel.
#include "rollout_kernel.h"

namespace gm {

KFn pick_kernel_het(int AW, int W, bool wg, int cut, bool probe)
{
    return pick_kernel_t<true, 0>(AW, W, wg, cut, probe);
}

}  // namespace gm
