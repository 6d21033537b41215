// Placeholder entry points, replaced by the batched and serving engines.
#include "internal.h"

using namespace di;

extern "C" {

di_status di_server_create(const di_server_opts*, di_server**) {
  set_error("server: not built yet");
  return DI_EINVAL;
}
di_status di_server_add_graph(di_server*, const di_graph*, int32_t*) { return DI_EINVAL; }
di_status di_server_submit(di_server*, int32_t, int32_t, const int32_t*, const double*, double,
                           double, uint64_t*) { return DI_EINVAL; }
di_status di_server_poll(di_server*, uint64_t, di_result*) { return DI_EINVAL; }
di_status di_server_wait(di_server*, uint64_t, double, di_result*) { return DI_EINVAL; }
di_status di_server_cancel(di_server*, uint64_t) { return DI_EINVAL; }
di_status di_server_stats(di_server*, di_server_metrics*) { return DI_EINVAL; }
di_status di_server_destroy(di_server*) { return DI_EINVAL; }
}
