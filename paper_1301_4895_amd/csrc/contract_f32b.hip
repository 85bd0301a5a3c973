// Recursion-step kernels (contract_impl.h) instantiated for float stages that
// read float copies of the block entries (MB_MIXED_F32B), sink base sets of
// up to four indices.
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f32b(const StageArgs &a, hipStream_t s) {
  if (a.M > 4) return hipErrorInvalidValue;   // no float-block kernels for three sources
  return launch_stage_t<float, float, 1, 4>(a, s);
}

}  // namespace mb
