// Kernel instantiations for compute type float with bf16 state storage.
#include "pf_launch.h"

namespace pfk {
hipError_t launch_bf16(const LaunchReq& rq, const void* args, hipStream_t st) {
  return launch_any<float, bf16>(rq, args, st);
}
}  // namespace pfk
