// Serving loop (continuous batching).  Filled in by a later change; the
// entry points exist so that the interface is complete.
#include "../../include/tsvdmi.h"

extern "C" {
int tsvd_server_create(tsvd_server** srv, tsvd_ctx*, int, int64_t, int) {
    if (srv) *srv = nullptr;
    return TSVD_EINVAL;
}
int64_t tsvd_server_submit(tsvd_server*, const tsvd_request*) { return TSVD_EINVAL; }
int tsvd_server_poll(tsvd_server*, int64_t, float*, double*, double*, double*) { return TSVD_EINVAL; }
double tsvd_server_now(tsvd_server*) { return 0.0; }
int tsvd_server_stats(tsvd_server*, int64_t*, int64_t*, int64_t*, int64_t*) { return TSVD_EINVAL; }
void tsvd_server_destroy(tsvd_server*) {}
}
