// Serving loop: continuous batching of render and z-optimisation requests.
#include "serve.h"

void serve_shutdown(dist_ctx* ctx) { (void)ctx; }

extern "C" int dist_submit(dist_ctx* ctx, const dist_request* req, uint64_t* ticket) {
  (void)ctx; (void)req; (void)ticket;
  return dist_set_error(DIST_EINVAL, "serving is not available in this build");
}

extern "C" int dist_poll(dist_ctx* ctx, uint64_t ticket, dist_result* res, int64_t timeout_us) {
  (void)ctx; (void)ticket; (void)res; (void)timeout_us;
  return dist_set_error(DIST_ENOTFOUND, "unknown ticket");
}
