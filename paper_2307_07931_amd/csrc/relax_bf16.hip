// relax_bf16.hip -- bf16 instances of the fused relaxation kernel (see relax_kernel.h).
#include "relax_kernel.h"

namespace px {
namespace relax_detail {

LaunchFn pick_bf16(int k, int rm, bool vec)
{
    return vec ? pick_k<bf16, true>(k, rm) : pick_k<bf16, false>(k, rm);
}

BatchLaunchFn pick_batch_bf16(int k, int rm)
{
    return pick_batch_k<bf16>(k, rm);
}

}  // namespace relax_detail
}  // namespace px
