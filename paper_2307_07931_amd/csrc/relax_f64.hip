// relax_f64.hip -- double instances of the fused relaxation kernel (see relax_kernel.h).
#include "relax_kernel.h"

namespace px {
namespace relax_detail {

LaunchFn pick_f64(int k, int rm, bool vec)
{
    return vec ? pick_k<double, true>(k, rm) : pick_k<double, false>(k, rm);
}

BatchLaunchFn pick_batch_f64(int k, int rm)
{
    return pick_batch_k<double>(k, rm);
}

}  // namespace relax_detail
}  // namespace px
