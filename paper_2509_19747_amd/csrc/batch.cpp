// Batched solves: several right-hand sides / shifts against one handle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ctx.hpp"

using namespace rr;

// Column-at-a-time driver: each column runs its own PCG recurrence with the
// handle's shared basis.
rr_status rr_solve_batch_fused(const rr_precond* P, const int32_t* mu_index_per_col,
                               const double* B, int64_t ldb, int32_t nrhs, double* X, int64_t ldx,
                               const rr_solve_opts* o, rr_solve_info* infos, void* hip_stream) {
    rr_status first = RR_OK;
    for (int32_t j = 0; j < nrhs; ++j) {
        rr_solve_info inf{};
        const rr_status s = rr_solve(P, mu_index_per_col[j], B + (size_t)j * ldb,
                                     X + (size_t)j * ldx, o, &inf, hip_stream);
        if (infos) infos[j] = inf;
        if (s != RR_OK && first == RR_OK) first = s;
        if (s == RR_EDEVICE || s == RR_EINVAL) return s;
    }
    return first;
}
