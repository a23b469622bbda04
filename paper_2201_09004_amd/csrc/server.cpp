// Serving loop (continuous batching) -- entry points.
#include "lq_internal.h"

using namespace lq;

extern "C" {

lq_status lq_server_create(lq_ctx* c, size_t hbm_budget, int max_cols, lq_server** srv) {
  (void)c; (void)hbm_budget; (void)max_cols; (void)srv;
  return (lq_status)fail(LQ_ENOTSUP, "server not available in this build");
}
lq_status lq_server_destroy(lq_server* srv) {
  (void)srv;
  return (lq_status)fail(LQ_ENOTSUP, "server not available in this build");
}
lq_status lq_submit(lq_server* srv, const lq_action* act, const lq_field* g, const lq_params* prm, int n_rhs,
                    const double* b, double* x, lq_stats* st, uint64_t* ticket) {
  (void)srv; (void)act; (void)g; (void)prm; (void)n_rhs; (void)b; (void)x; (void)st; (void)ticket;
  return (lq_status)fail(LQ_ENOTSUP, "server not available in this build");
}
lq_status lq_poll(lq_server* srv, uint64_t ticket, int* done) {
  (void)srv; (void)ticket; (void)done;
  return (lq_status)fail(LQ_ENOTSUP, "server not available in this build");
}
lq_status lq_wait(lq_server* srv, uint64_t ticket) {
  (void)srv; (void)ticket;
  return (lq_status)fail(LQ_ENOTSUP, "server not available in this build");
}
lq_status lq_server_stats(lq_server* srv, double* p50, double* p99, double* sps) {
  (void)srv; (void)p50; (void)p99; (void)sps;
  return (lq_status)fail(LQ_ENOTSUP, "server not available in this build");
}

}  // extern "C"
