// Grouped PCG iterations of many kernel ridge solves (the serving loop).
//
// One grouped iteration advances every column of every submitted request by one
// C-RandRAND PCG step (Algorithm RandRAND_PCG, step 8) with one launch per kernel
// kind for all of them, instead of one launch per request:
//   kernel product W = A_mu P   per column block       (GL_MAT + (kind, record length, width))
//   its finish                   per column block       (GL_FIN)
//   alpha, x, r, ||r||^2          per request            (GL_BXR)
//   C = Q^T R                    per column group       (GL_GEMV + width)
//   D = Kc C                     per column group       (GL_CORE)
//   Z = R + Q D, r^T z           per column group       (GL_QD + width)
//   beta, p                      per request            (GL_BP)
// A request's work items are the same blocks, in the same layout, as its own
// launches would be (the shared block bodies of kernels_ksym_mma.hip,
// kernels_blas.hip and kernels_batch.hip), and every reduction keeps its fixed
// order, so each result is bitwise independent of the other requests in the group.
//
// The host writes the unit arrays and list headers before each replay; the kernels
// are persistent: each block takes work items from its list's counter until the list
// is exhausted.  Units whose columns have all stopped are skipped (their run flags).
#pragma once
#include <cstdint>

#include "../../include/randrand.h"
#include "common.hpp"
#include "kernels.hpp"

namespace rr {

enum GroupListId {
    GL_MAT = 0,    // + 12 (kind - 1) + 3 record class (dm 4, 8, 16, 32) + width class (1, 2, 4)
    GL_FIN = 24,
    GL_BXR,
    GL_GEMV,       // + width class (1, 2, 4, 8 columns): 4 lists
    GL_CORE = GL_GEMV + 4,
    GL_QD,         // + width class: 4 lists
    GL_BP = GL_QD + 4,
    GL_COUNT
};

// Units [off, off + count) of the list's unit array; total = work items of the list.
struct GList {
    int32_t off, count, total, pad;
};

// One block of nr consecutive columns of one request (nr = 1, 2 or 4; the last
// nr - ncols are zero padding): the kernel product and its finish.
struct GPair {
    const float* xa;
    const float* sqn;
    const double* u;        // nr columns, leading dimension n
    double* part;           // slot partials of the block
    double* y;              // nr columns
    double* dot;            // finish partials of u^T y: nr columns of nfb
    const BState* st;       // the block's column states
    int64_t n;
    double scale, mu;
    float c;
    int32_t nr, ncols;
    int32_t nb, m, S;       // work-item plan of the product
    int32_t nfb;            // finish blocks
    int32_t w_mat, w_fin;   // first work item within the GL_MAT and GL_FIN lists
    int32_t pad;
};

// One request: the fused x, r and p updates of its m columns.
struct GVec {
    int64_t n, ldx;
    double* X;
    double* R;
    double* P;
    const double* W;
    const double* Z;
    BState* st;
    ColParts pw, rz;        // block partials of p^T w and r^T z
    double* rr_part;
    int32_t* cnt;           // 2 m block counters (x/r update, p update)
    int32_t m, nbx;
    int32_t w0;             // first work item within GL_BXR (and GL_BP)
    int32_t pad;
};

// One group of nr consecutive columns of a request: the projection through the basis.
struct GProj {
    int64_t n, k;
    const double* Q;        // n x k, leading dimension n
    const double* Kc;       // k x k core
    const double* R;        // nr columns, leading dimension n
    double* cpart;          // nr x nch x k partials of Q^T R
    double* D;              // nr x k
    double* Z;              // nr columns, leading dimension n
    double* rz;             // nr x nbq partials of r^T z
    const BState* st;       // the group's column states
    int64_t rpc;            // rows per chunk of Q^T R
    int32_t nr, nch, cblk, nbq;
    int32_t w_gemv, w_core, w_qd;
    int32_t pad;
};

// Device-side list headers and work counters of one replay (iters iterations).
struct GTable {
    GList list[GL_COUNT];
};

constexpr int GROUP_COUNTERS_PER_ITER = GL_COUNT;
// Largest core dimension k of a projection group of nr columns (its D lives in LDS).
constexpr int64_t group_qd_kmax(int nr) { return nr >= 8 ? 768 : 1792; }

int group_rec_class(int dm);     // 0..3 for record lengths 4, 8, 16, 32
int group_width_class(int nr);   // 0..3 for 1, 2, 4, 8 columns
int group_mat_list(int kind, int dm, int nr);   // the GL_MAT list of a column block

// Launch the kernels of one list: a persistent grid of at most group_list_blocks(list)
// blocks (fewer when the list has fewer work items), work from counter ctr.
int group_list_blocks(int list);
void launch_group_list(int list, int blocks, const GTable* tab, const GPair* pairs, const GVec* vecs,
                       const GProj* projs, int32_t* ctr, hipStream_t st);
// Zero ncount work counters (the first node of a replay).
void launch_group_reset(int32_t* ctr, int ncount, hipStream_t st);
// Per-file launchers behind launch_group_list.
void launch_group_mat(int list, int blocks, const GTable* tab, const GPair* pairs, int32_t* ctr, hipStream_t st);
void launch_group_fin(int blocks, const GTable* tab, const GPair* pairs, int32_t* ctr, hipStream_t st);
void launch_group_vec(bool bp, int blocks, const GTable* tab, const GVec* vecs, int32_t* ctr, hipStream_t st);
void launch_group_proj(int list, int blocks, const GTable* tab, const GProj* projs, int32_t* ctr, hipStream_t st);
// Persistent grid caps: two blocks per compute unit for the products and Q^T R / core
// stages, one for the finish, the vector updates and Z = R + Q D (their lists are
// short, and blocks that find the list drained still cost a dispatch).
constexpr int GROUP_MAT_BLOCKS = 512, GROUP_FIN_BLOCKS = 256, GROUP_VEC_BLOCKS = 256,
              GROUP_PROJ_BLOCKS = 512, GROUP_QD_BLOCKS = 256;

// ------------------------------------------------------------ host engine
struct Batch;
struct GroupStats {
    int64_t replays, jobs, max_jobs;   // replays, request batches they carried, largest group
    double busy_s;                     // wall time from each replay's upload to its completion (summed over lanes)
    double wait_s;                     // summed over request batches: queued until completed
};
// One engine per serving loop: iters grouped iterations per replay, at most max_jobs
// requests per replay, `lanes` replays in flight at once (each on its own stream).
// run() blocks the calling worker until a replay that included its column block has
// completed.
class GroupEngine {
  public:
    GroupEngine(int iters, int max_jobs, int lanes);
    ~GroupEngine();
    GroupEngine(const GroupEngine&) = delete;
    GroupEngine& operator=(const GroupEngine&) = delete;
    rr_status init();   // device buffers and the engine thread (throws on failure)
    rr_status run(Batch& bt, double* X, int64_t ldx);
    GroupStats stats();

  private:
    struct Impl;
    Impl* impl_;
};

// ------------------------------------------------------------ device helpers
// Value made wave-uniform (held in scalar registers by the code that uses it).
RR_DEV int32_t gu(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
RR_DEV int64_t gu(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
RR_DEV double gu(double v) { return __builtin_bit_cast(double, gu(__builtin_bit_cast(int64_t, v))); }
RR_DEV float gu(float v) { return __builtin_bit_cast(float, gu(__builtin_bit_cast(int32_t, v))); }
template <typename T>
RR_DEV T* gu(T* p) { return reinterpret_cast<T*>(gu((int64_t)reinterpret_cast<uintptr_t>(p))); }

// Work items of a persistent block: thread 0 takes them from the list's counter one
// item ahead, so the atomic's round trip overlaps the current item.  next() starts
// with a barrier that ends the previous item (its LDS and *sh are free again).
struct GroupCursor {
    int32_t* ctr;
    int32_t* sh;       // one LDS word
    int32_t ahead = 0; // thread 0: the item taken for the next call
    RR_DEV GroupCursor(int32_t* c, int32_t* s) : ctr(c), sh(s) {
        if (threadIdx.x == 0) ahead = atomicAdd(ctr, 1);
    }
    RR_DEV int32_t next() {
        __syncthreads();
        if (threadIdx.x == 0) {
            *sh = ahead;
            ahead = atomicAdd(ctr, 1);
        }
        __syncthreads();
        return gu(*sh);
    }
};

// Unit of work item w in units [lo, hi): the last one whose first item first(u) <= w.
template <typename U, typename F>
RR_DEV int32_t group_find(const U* __restrict__ units, int32_t lo, int32_t hi, int32_t w, F first) {
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (gu(first(units[mid])) <= w) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace rr
