// Kernel instantiations of the batched filters (FP32 states and weights).
#include "pf_launch.h"

namespace pfk {
hipError_t launch_batch(const BatchReq& rq, const BatchArgs& a, hipStream_t st) {
  if (rq.mk == MK_SV) return rq.D == 1 ? launch_batch_model<1, MK_SV>(rq, a, st) : hipErrorInvalidValue;
#define PFK_BATCH_DIMS(MKV)                                           \
  switch (rq.D) {                                                     \
    case 1: return launch_batch_model<1, MKV>(rq, a, st);             \
    case 2: return launch_batch_model<2, MKV>(rq, a, st);             \
    case 4: return launch_batch_model<4, MKV>(rq, a, st);             \
    case 8: return launch_batch_model<8, MKV>(rq, a, st);             \
    case 16: return launch_batch_model<16, MKV>(rq, a, st);           \
    default: return hipErrorInvalidValue;                             \
  }
  if (rq.mk == MK_LG_DENSE) { PFK_BATCH_DIMS(MK_LG_DENSE) }
  if (rq.mk == MK_LG_DIAG) { PFK_BATCH_DIMS(MK_LG_DIAG) }
#undef PFK_BATCH_DIMS
  return hipErrorInvalidValue;
}
}  // namespace pfk
