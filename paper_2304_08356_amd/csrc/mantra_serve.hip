// Serving scheduler (continuous batching of progressive-sampling rounds).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/mantra.h"

extern "C" {
int mantra_serve_stop(mantra_graph *g) { (void)g; return MANTRA_OK; }
int mantra_serve_config(mantra_graph *g, uint64_t mem_budget_bytes, int32_t max_active) {
    (void)g; (void)mem_budget_bytes; (void)max_active; return MANTRA_E_INTERNAL;
}
int mantra_submit(mantra_graph *g, const mantra_request *req, uint64_t *ticket) {
    (void)g; (void)req; (void)ticket; return MANTRA_E_INTERNAL;
}
int mantra_poll(uint64_t ticket, mantra_result *out, int32_t timeout_ms) {
    (void)ticket; (void)out; (void)timeout_ms; return MANTRA_E_INTERNAL;
}
}
