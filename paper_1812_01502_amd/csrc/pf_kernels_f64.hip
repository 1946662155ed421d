// Kernel instantiations for compute type double with double state storage.
#include "pf_launch.h"

namespace pfk {
hipError_t launch_f64(const LaunchReq& rq, const void* args, hipStream_t st) {
  return launch_any<double, double>(rq, args, st);
}
}  // namespace pfk
