// Incremental update (Sec. IV-D) -- placeholder until the GPU update kernels land.
#include "cddt_common.h"

namespace cddt {
cddt_status apply_update(cddt_map_s*, const int32_t*, const int32_t*, const uint8_t*, int64_t, hipStream_t) {
  return fail(CDDT_EINTERNAL, "cddt_update: not available in this build");
}
}  // namespace cddt
