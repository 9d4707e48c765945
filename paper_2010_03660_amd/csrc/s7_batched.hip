// Batched solves (placeholder until the persistent driver lands).
#include "s7_host.hpp"

extern "C" {
size_t s7_batched_workspace_bytes(int32_t, const s7_dims*, int32_t, const s7_options*) { return 0; }
int s7_bicgstab_solve_batched(int32_t, const s7_dims*, const float* const*, const double* const*,
                              double* const*, const double*, const int32_t*, int32_t, void*, size_t,
                              const s7_options*, s7_info*, void*) {
    s7::set_error("not implemented");
    return S7_EINVAL;
}
int s7_queue_create(s7_queue**, void*, size_t, const s7_options*) { return S7_EINVAL; }
int s7_queue_submit(s7_queue*, const s7_request*, uint64_t*) { return S7_EINVAL; }
int s7_queue_poll(s7_queue*, uint64_t, s7_info*) { return S7_EINVAL; }
int s7_queue_wait(s7_queue*, uint64_t, s7_info*) { return S7_EINVAL; }
int s7_queue_destroy(s7_queue*) { return S7_EINVAL; }
}
