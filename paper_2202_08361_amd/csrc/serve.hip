// serve.hip -- continuous-batching SVD server (to be completed).
#include <hip/hip_runtime.h>

#include "../../include/jsvd.h"

extern "C" int jsvd_serve_create(const jsvd_serve_config *, jsvd_server *out)
{
    if (out) *out = nullptr;
    return JSVD_EINVAL;
}
extern "C" int jsvd_serve_submit(jsvd_server, const jsvd_request *, uint64_t *) { return JSVD_EINVAL; }
extern "C" int jsvd_serve_poll(jsvd_server, uint64_t, int *, int *, int *) { return JSVD_EINVAL; }
extern "C" int jsvd_serve_wait(jsvd_server, uint64_t, int *, int *) { return JSVD_EINVAL; }
extern "C" int jsvd_serve_stats_get(jsvd_server, jsvd_serve_stats *) { return JSVD_EINVAL; }
extern "C" int jsvd_serve_destroy(jsvd_server) { return JSVD_EINVAL; }
