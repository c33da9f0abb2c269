// Serving: continuous batching of solve requests.
#include "qs3_impl.h"

using namespace qs3;

extern "C" {
int qs3_server_create(qs3_ctx *, const qs3_server_opts *, qs3_server **) { set_error("not built yet"); return QS3_EINVAL; }
int qs3_server_destroy(qs3_server *) { return QS3_OK; }
int qs3_submit(qs3_server *, const qs3_request *, uint64_t *) { set_error("not built yet"); return QS3_EINVAL; }
int qs3_poll(qs3_server *, uint64_t, qs3_result *) { return QS3_ENOTFOUND; }
int qs3_wait(qs3_server *, uint64_t, qs3_result *) { return QS3_ENOTFOUND; }
int qs3_cancel(qs3_server *, uint64_t) { return QS3_ENOTFOUND; }
double qs3_server_clock(qs3_server *) { return 0.0; }
}
