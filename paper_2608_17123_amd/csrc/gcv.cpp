// GCV driver (placeholder until the GCV kernels land).
#include "runtime.h"

namespace dbl {
int gcv_run(dbl_ctx* ctx, std::vector<GcvReq>&) {
  return set_err(ctx, DBL_ENOTSUP, "GCV not built yet");
}
}  // namespace dbl
