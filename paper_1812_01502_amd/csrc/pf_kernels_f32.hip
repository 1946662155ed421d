// Kernel instantiations for compute type float with float state storage.
#include "pf_launch.h"

namespace pfk {
hipError_t launch_f32(const LaunchReq& rq, const void* args, hipStream_t st) {
  if (rq.what == LW_STEP_TILE && rq.full) return launch_f32_full(rq, args, st);
  return launch_any<float, float>(rq, args, st);
}
}  // namespace pfk
