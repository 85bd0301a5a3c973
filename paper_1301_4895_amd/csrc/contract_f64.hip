// Recursion-step kernels (contract_impl.h) instantiated for double stages.
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f64(const StageArgs &a, hipStream_t s) { return launch_stage_t<double>(a, s); }
hipError_t launch_stage_lds_f64(const StageLdsArgs &a, hipStream_t s) { return launch_stage_lds_t<double>(a, s); }

}  // namespace mb
