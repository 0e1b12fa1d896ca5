// Serving loop -- placeholder.
#include "cddt_common.h"
using namespace cddt;
extern "C" {
cddt_status cddt_server_create(const cddt_map*, int32_t, const float* const*, const int32_t*, const float* const*,
                               const int32_t*, const cddt_server_config*, cddt_server*) {
  return fail(CDDT_EINTERNAL, "server not available in this build");
}
cddt_status cddt_server_submit(cddt_server, int32_t, const float*, const float*, const float*, int32_t,
                               const int32_t*, int64_t*) { return CDDT_EINTERNAL; }
cddt_status cddt_server_poll(cddt_server, int64_t, float*, int32_t*) { return CDDT_EINTERNAL; }
cddt_status cddt_server_wait(cddt_server, int64_t, float*) { return CDDT_EINTERNAL; }
cddt_status cddt_server_times(cddt_server, int64_t, double*, double*) { return CDDT_EINTERNAL; }
cddt_status cddt_server_stats_get(cddt_server, cddt_server_stats*) { return CDDT_EINTERNAL; }
double cddt_server_now(cddt_server) { return 0.0; }
cddt_status cddt_server_destroy(cddt_server) { return CDDT_OK; }
}
