// Event-based tracking (placeholder until the queue kernels land).
#include "k_common.hpp"

namespace mcdc {

int launch_event(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count,
                 const mcdc_run_options &opt, hipStream_t st) {
    (void)p; (void)R; (void)first; (void)count; (void)opt; (void)st;
    set_error("event-based algorithm not built yet");
    return MCDC_E_UNSUPPORTED;
}

}  // namespace mcdc
