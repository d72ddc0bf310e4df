// Serving runtime (placeholder until the incremental path lands).
#include <hip/hip_runtime.h>

#include "hpop.h"

struct hpop_server {
  int unused;
};

extern "C" {
hpop_status hpop_server_create(const hpop_server_config*, hpop_server** out) {
  if (out) *out = nullptr;
  return HPOP_E_STATE;
}
hpop_status hpop_server_destroy(hpop_server*) { return HPOP_E_STATE; }
hpop_status hpop_server_open_session(hpop_server*, int32_t, int32_t, int64_t, int32_t*) { return HPOP_E_STATE; }
hpop_status hpop_server_submit(hpop_server*, int32_t, const hpop_event_chunk*, int32_t, int32_t, int64_t, int64_t,
                               uint64_t*) {
  return HPOP_E_STATE;
}
hpop_status hpop_server_wait(hpop_server*, uint64_t, int64_t, hpop_metric_tree*, hpop_metric_tree*) {
  return HPOP_E_STATE;
}
hpop_status hpop_server_get_stats(hpop_server*, hpop_server_stats*) { return HPOP_E_STATE; }
const char* hpop_server_last_error(const hpop_server*) { return "serving runtime not built"; }
}
