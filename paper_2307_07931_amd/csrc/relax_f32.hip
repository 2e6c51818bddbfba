// relax_f32.hip -- float instances of the fused relaxation kernel (see relax_kernel.h).
#include "relax_kernel.h"

namespace px {
namespace relax_detail {

LaunchFn pick_f32(int k, int rm, bool vec)
{
    return vec ? pick_k<float, true>(k, rm) : pick_k<float, false>(k, rm);
}

BatchLaunchFn pick_batch_f32(int k, int rm)
{
    return pick_batch_k<float>(k, rm);
}

}  // namespace relax_detail
}  // namespace px
