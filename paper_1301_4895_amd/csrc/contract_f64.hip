// Recursion-step kernels (contract_impl.h) instantiated for double stages and
// sink base sets of up to four indices; contract_f64_m6.hip holds five and six.
#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f64_m6(const StageArgs &a, hipStream_t s);

hipError_t launch_stage_f64(const StageArgs &a, hipStream_t s) {
  return a.M <= 4 ? launch_stage_t<double, double, 1, 4>(a, s) : launch_stage_f64_m6(a, s);
}
hipError_t launch_stage_lds_f64(const StageLdsArgs &a, hipStream_t s) { return launch_stage_lds_t<double>(a, s); }

}  // namespace mb
