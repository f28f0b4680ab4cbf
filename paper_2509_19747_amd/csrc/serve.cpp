// Continuous-batching serving loop (placeholder until the server lands).
#include "ctx.hpp"

using namespace rr;

extern "C" rr_status rr_serve(const rr_serve_config* cfg, rr_next_fn next, rr_deliver_fn deliver,
                              void* user, rr_serve_stats* stats) {
    (void)cfg; (void)next; (void)deliver; (void)user; (void)stats;
    set_error("rr_serve is not available in this build");
    return RR_EINVAL;
}
