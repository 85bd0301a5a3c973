// Recursion-step kernels (contract_impl.h) instantiated for float stages.
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f32(const StageArgs &a, hipStream_t s) { return launch_stage_t<float>(a, s); }
hipError_t launch_stage_lds_f32(const StageLdsArgs &a, hipStream_t s) { return launch_stage_lds_t<float>(a, s); }

}  // namespace mb
