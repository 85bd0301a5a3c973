// Recursion-step kernels (contract_impl.h) instantiated for float stages that
// read float copies of the block entries (MB_MIXED_F32B), sink base sets of
// up to four indices; contract_f32b_m6.hip holds five and six.
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f32b_m6(const StageArgs &a, hipStream_t s);

hipError_t launch_stage_f32b(const StageArgs &a, hipStream_t s) {
  return a.M <= 4 ? launch_stage_t<float, float, 1, 4>(a, s) : launch_stage_f32b_m6(a, s);
}

}  // namespace mb
