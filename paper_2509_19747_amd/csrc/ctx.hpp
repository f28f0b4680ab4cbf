// Host-side internals shared by the C-ABI entry points: error reporting,
// device allocations, the preconditioner handle and the operator dispatch.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/randrand.h"
#include "kernels.hpp"

namespace rr {

void set_error(const std::string& msg);
const std::string& last_error();

struct RrError {
    rr_status st;
    std::string msg;
};

#define RR_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            throw ::rr::RrError{RR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
        }                                                                              \
    } while (0)

#define RR_REQUIRE(cond, msg)                                           \
    do {                                                                \
        if (!(cond)) throw ::rr::RrError{RR_EINVAL, std::string(msg)};  \
    } while (0)

// Run `body`, translating exceptions to status codes; never lets one escape.
template <typename F>
rr_status guarded(F&& body) {
    try {
        return body();
    } catch (const RrError& e) {
        set_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return RR_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return RR_EDEVICE;
    }
}

// Device allocator: the caller's rr_allocator if given, else hipMalloc/hipFree.
// Frees the blocks the allocator cache holds for stream st (on this device) and
// forgets the stream: called before the library destroys a stream it created.
void release_stream_blocks(hipStream_t st);

struct Alloc {
    rr_allocator a{};
    bool custom = false;
    hipStream_t st = nullptr;
    void* get(size_t bytes) const;
    void put(void* p) const;
};

// Non-blocking streams (each with two timing-free events) kept in a process-wide
// pool per device and reused: the library never creates or destroys a stream
// inside a build or a solve, so concurrent requests do not churn streams while
// other threads capture graphs.
struct SideStream {
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int dev = 0;
};
SideStream acquire_side_stream();
void release_side_stream(const SideStream& s);
class PooledStream {
  public:
    PooledStream() = default;
    ~PooledStream() { reset(); }
    PooledStream(const PooledStream&) = delete;
    PooledStream& operator=(const PooledStream&) = delete;
    hipStream_t get() {
        if (!s_.st) s_ = acquire_side_stream();
        return s_.st;
    }
    hipEvent_t ev_a() { get(); return s_.a; }
    hipEvent_t ev_b() { get(); return s_.b; }
    bool active() const { return s_.st != nullptr; }
    hipStream_t raw() const { return s_.st; }
    void reset() {
        if (s_.st) {
            (void)hipStreamSynchronize(s_.st);
            release_side_stream(s_);
            s_ = SideStream{};
        }
    }

  private:
    SideStream s_;
};

// Owning device buffer.
class DBuf {
  public:
    DBuf() = default;
    DBuf(const Alloc* al, size_t bytes) { reset(al, bytes); }
    ~DBuf() { release(); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept { *this = std::move(o); }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            release();
            al_ = o.al_; p_ = o.p_; bytes_ = o.bytes_;
            o.p_ = nullptr; o.bytes_ = 0;
        }
        return *this;
    }
    void reset(const Alloc* al, size_t bytes) {
        release();
        al_ = al;
        bytes_ = bytes;
        p_ = bytes ? al->get(bytes) : nullptr;
    }
    void release() {
        if (p_ && al_) al_->put(p_);
        p_ = nullptr;
        bytes_ = 0;
    }
    template <typename T> T* as() const { return (T*)p_; }
    void* ptr() const { return p_; }
    size_t bytes() const { return bytes_; }

  private:
    const Alloc* al_ = nullptr;
    void* p_ = nullptr;
    size_t bytes_ = 0;
};

inline double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Per-shift state of a handle: the apply core Kc over the basis Qb, plus the
// l x l factors kept for inspection.
struct PerMu {
    double mu = 0.0;
    DBuf Kc;        // kb x kb: P = I + Qb Kc Qb^T
    DBuf R, G, T;   // l x l
    DBuf Qred;      // 2l x l (joint basis only)
    double tau = 1.0, normE = 0.0, lam = 0.0;
};

struct Workspace;

}  // namespace rr

void rr_free_workspace(rr::Workspace* w);
void rr_workspace_null_stream(rr::Workspace* w);   // free on the null stream from now on
// Release a handle whose work has completed.  keep_stream: its blocks stay in the
// allocator cache of the stream it was built on (the caller guarantees that stream
// is alive, as the server's worker streams are); otherwise they go to the null
// stream's cache.
void rr_precond_release(rr_precond* P, bool keep_stream);

struct rr_precond {
    rr_operator op{};
    rr_build_opts opts{};
    int64_t n = 0, l = 0, kb = 0;   // kb: columns of the apply basis (l or 2l)
    bool joint = false;
    rr::Alloc alloc;
    // operator-derived data
    rr::DBuf A32;         // float32 copy of a dense A (FP32 / MIXED)
    rr::DBuf sqn;         // |x_i|^2 (kernel operators)
    rr::DBuf xa;          // padded point records (kernel operators)
    rr::DBuf xd, hd;      // float64 point records and -g |x_i|^2 / 2 (kernel operators)
    // basis
    rr::DBuf Omega;       // n x l, dtype omega_dt
    int omega_dt = rr::DT_F64;
    rr::DBuf Qb;          // n x kb float64 (not stored by a basis-less handle)
    // basis-less handle (signed column sampling): Omega's columns sgn_c e_idx_c,
    // pos[i] = c for i = idx_c (else -1); Q = A_mu Omega R^{-1} is never formed
    bool basisless = false;
    rr::DBuf bl_idx, bl_sgn, bl_pos;
    std::vector<rr::PerMu> per;
    double orth_err = 0.0;
    double ms_build = 0.0;
    int device = 0;
    // solve workspaces: each rr_solve takes one from this pool (or makes one) and
    // returns it, so concurrent solves on one handle run with their own
    // workspaces; the pool is guarded by ws_mu
    std::mutex ws_mu;
    std::vector<rr::Workspace*> ws_pool;
    ~rr_precond();
};

namespace rr {

// Working-precision helpers.
inline bool is_kernel(const rr_operator& op) { return op.kind == RR_OP_RBF || op.kind == RR_OP_MATERN32; }

KernelOp kernel_op_of(const rr_precond& P);

// y = (A + mu I) u with dot partials of u^T y; returns the number of partials.
// fp64 = use the float64 operator (dense A or float64 kernel entries).
int apply_operator(const rr_precond& P, const double* u, double mu, double* y, double* dot_part,
                   double* kmv_ws, bool fp64, const int32_t* stop, hipStream_t st);
// Same for nr (1 or 2) columns U, Y (n x nr); dot partials of column q start at
// dot_part + q * operator_part_count(P).
// Several columns at once; estimate: float32 sums allowed for kernel operators in
// float32 mode (the power iterations of the tau estimates).
void apply_operator_multi(const rr_precond& P, const double* U, int nr, double mu, double* Y,
                          double* dot_part, double* kmv_ws, bool fp64, hipStream_t st,
                          bool estimate = false);
int operator_part_count(const rr_precond& P);
// Operator setup (A0): squared norms and point records for kernels, the float32
// copy of a dense A when the working precision is below float64.
void setup_operator(rr_precond& P, hipStream_t st);
size_t operator_ws_doubles(const rr_precond& P);

// z = rcoef*r + Qb (Kc (Qb^T r)), with partials of r^T z.  Returns #partials.
int apply_projected(const rr_precond& P, const double* Kc, const double* r, double rcoef, double* z,
                    double* c_part, double* d, double* rz_part, const int32_t* stop, hipStream_t st);
// Two vectors at once (R, Z: n x 2, leading dimension n), each with its own core:
// Z[:, q] = rc_q R[:, q] + Q K_q Q^T R[:, q].  c_part: 2 * nchunks * kb doubles,
// d: 2 * kb, rz_part: 2 * qd_blocks(n).
void apply_projected_pair(const rr_precond& P, const double* K0, const double* K1, const double* R,
                          double rc0, double rc1, double* Z, double* c_part, double* d,
                          double* rz_part, hipStream_t st);

rr_status validate_operator(const rr_operator* A);
void require_device();

struct BatchRunner;
// rr_solve_batch (argument checks included) with a runner for its iteration batches.
rr_status solve_batch_with(const rr_precond* P, const int32_t* mu_index_per_col, const double* B,
                           int64_t ldb, int32_t nrhs, double* X, int64_t ldx, const rr_solve_opts* opts,
                           rr_solve_info* infos, void* hip_stream, BatchRunner* runner);

}  // namespace rr

// runner: where the column block's PCG iteration batches run (the serving loop's
// grouped replays), nullptr for the solve's own launches or hipGraph.
rr_status rr_solve_batch_fused(const rr_precond* P, const int32_t* mu_index_per_col,
                               const double* B, int64_t ldb, int32_t nrhs, double* X, int64_t ldx,
                               const rr_solve_opts* o, rr_solve_info* infos, void* hip_stream,
                               rr::BatchRunner* runner = nullptr);
rr_status rr_solve_block(const rr_precond* P, const int32_t* mu_index_per_col, const double* B, int64_t ldb,
                         int32_t nrhs, double* X, int64_t ldx, const rr_solve_opts* o, rr_solve_info* infos,
                         void* hip_stream);
