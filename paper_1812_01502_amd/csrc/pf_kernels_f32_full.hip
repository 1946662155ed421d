// Step-kernel instantiations for FP32 states when the model dimension equals
// the compiled one (every benchmarked workload).
#include "pf_launch.h"

namespace pfk {
hipError_t launch_f32_full(const LaunchReq& rq, const void* args, hipStream_t st) {
  return launch_full_any<float, float>(rq, args, st);
}
}  // namespace pfk
