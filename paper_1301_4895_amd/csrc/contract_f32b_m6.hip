// Recursion-step kernels (contract_impl.h) instantiated for float stages that
// read float copies of the block entries (MB_MIXED_F32B), sink base sets of
// five or six indices (three quark sources).
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f32b_m6(const StageArgs &a, hipStream_t s) { return launch_stage_t<float, float, 5, 6>(a, s); }

}  // namespace mb
