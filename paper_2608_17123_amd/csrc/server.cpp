// Continuous-batching server (placeholder until the serving loop lands).
#include "runtime.h"

extern "C" {
int dbl_server_create(dbl_ctx* ctx, int, size_t, dbl_server** out) {
  if (out) *out = nullptr;
  return dbl::set_err(ctx, DBL_ENOTSUP, "server not built yet");
}
int dbl_server_destroy(dbl_server*) { return DBL_ENOTSUP; }
int dbl_server_submit(dbl_server*, const dbl_request*, int64_t*) { return DBL_ENOTSUP; }
int dbl_server_step(dbl_server*, int*) { return DBL_ENOTSUP; }
int dbl_server_poll(dbl_server*, int64_t, int*, dbl_report*) { return DBL_ENOTSUP; }
}
