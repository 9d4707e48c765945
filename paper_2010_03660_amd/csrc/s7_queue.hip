// Request queue (placeholder until the serving core lands).
#include "s7_host.hpp"

extern "C" {
int s7_queue_create(s7_queue**, void*, size_t, const s7_options*) { return S7_EINVAL; }
int s7_queue_submit(s7_queue*, const s7_request*, uint64_t*) { return S7_EINVAL; }
int s7_queue_poll(s7_queue*, uint64_t, s7_info*) { return S7_EINVAL; }
int s7_queue_wait(s7_queue*, uint64_t, s7_info*) { return S7_EINVAL; }
int s7_queue_destroy(s7_queue*) { return S7_EINVAL; }
}
