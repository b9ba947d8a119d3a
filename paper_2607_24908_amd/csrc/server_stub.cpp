// Placeholder until the flow server lands.
#include "frg_ctx.h"

namespace frg {
void Context::stop_server() {}
void Tune::load_env() {}
}  // namespace frg

extern "C" {
int frg_submit(frg_ctx *, const frg_request *, uint64_t *) {
  return frg::fail(FRG_E_INVAL, "flow server not available in this build");
}
int frg_poll(frg_ctx *, uint64_t, frg_result *) {
  return frg::fail(FRG_E_NOTFOUND, "flow server not available in this build");
}
int frg_server_stats(frg_ctx *, int64_t *, int64_t *, double *) {
  return frg::fail(FRG_E_INVAL, "flow server not available in this build");
}
}
