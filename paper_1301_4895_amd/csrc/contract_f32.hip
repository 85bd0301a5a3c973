// Recursion-step kernels (contract_impl.h) instantiated for float stages,
// double block entries and sink base sets of up to four indices;
// contract_f32_m6.hip holds five and six, contract_f32b.hip the float block
// entries.
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f32_m6(const StageArgs &a, hipStream_t s);

hipError_t launch_stage_f32(const StageArgs &a, hipStream_t s) {
  return a.M <= 4 ? launch_stage_t<float, double, 1, 4>(a, s) : launch_stage_f32_m6(a, s);
}
hipError_t launch_stage_lds_f32(const StageLdsArgs &a, hipStream_t s) { return launch_stage_lds_t<float>(a, s); }

}  // namespace mb
