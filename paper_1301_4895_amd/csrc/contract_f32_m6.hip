// Recursion-step kernels (contract_impl.h) instantiated for float stages and
// sink base sets of five or six indices (three quark sources).
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f32_m6(const StageArgs &a, hipStream_t s) { return launch_stage_t<float, double, 5, 6>(a, s); }

}  // namespace mb
