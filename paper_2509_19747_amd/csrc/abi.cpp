// C-ABI plumbing: error strings, defaults, allocation, operator dispatch,
// inspection/export entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace rr {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const std::string& last_error() { return g_last_error; }

// Without a caller allocator, buffers come from the device's stream-ordered
// pool (hipMallocAsync / hipFreeAsync on the Alloc's stream).  The pool keeps
// freed memory for reuse, so the many short-lived buffers of a build or a solve
// cost neither a device synchronisation (hipFree has one) nor a driver call.
static void keep_pool_memory() {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(mu);
    for (int d : done)
        if (d == dev) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();
    done.push_back(dev);
}

// On top of the pool, freed blocks are kept per (device, stream) and handed back
// to later requests on the same stream that they fit (at most 1/4 larger), so a
// build or a solve that repeats an earlier one's shapes makes no allocator call
// at all: pool calls right after a host synchronisation were measured at up to a
// millisecond each.  Reuse on the same stream is ordered after every earlier use.
// Each stream's cache holds at most kStreamCacheCap bytes (oldest blocks go back
// to the pool first); a failed pool allocation returns every cached block and
// retries once.
namespace {
struct CachedBlock {
    void* p;
    size_t bytes;
};
struct StreamCache {
    int dev;
    hipStream_t st;
    std::vector<CachedBlock> blocks;   // oldest first
    size_t total = 0;
};
constexpr size_t kStreamCacheCap = (size_t)4 << 30;
std::mutex g_cache_mu;
std::vector<StreamCache> g_caches;
std::vector<CachedBlock> g_live;   // blocks handed out by Alloc::get (pointer, size)

StreamCache& cache_for(int dev, hipStream_t st) {
    for (auto& c : g_caches)
        if (c.dev == dev && c.st == st) return c;
    g_caches.push_back(StreamCache{dev, st, {}, 0});
    return g_caches.back();
}

size_t round_block(size_t bytes) {
    const size_t g = bytes >= ((size_t)1 << 20) ? ((size_t)1 << 20) : 256;
    return (bytes + g - 1) / g * g;
}

void flush_all_caches() {   // caller holds g_cache_mu
    for (auto& c : g_caches) {
        // a stream that is being captured into a graph (by another thread) keeps its
        // blocks: a free queued on it would become part of, or break, that capture
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(c.st, &cs) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        if (cs != hipStreamCaptureStatusNone) continue;
        for (auto& b : c.blocks) (void)hipFreeAsync(b.p, c.st);
        c.blocks.clear();
        c.total = 0;
    }
}
}  // namespace

void* Alloc::get(size_t bytes) const {
    void* p = nullptr;
    if (custom) {
        p = a.alloc(a.ctx, bytes, (void*)st);
        if (!p) throw RrError{RR_ENOMEM, "allocator returned null for " + std::to_string(bytes) + " bytes"};
        return p;
    }
    keep_pool_memory();
    int dev = 0;
    (void)hipGetDevice(&dev);
    const size_t want = round_block(bytes);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    StreamCache& c = cache_for(dev, st);
    size_t best = SIZE_MAX, bi = 0;
    for (size_t i = 0; i < c.blocks.size(); ++i) {
        const size_t b = c.blocks[i].bytes;
        if (b >= want && b - want <= want / 4 && b < best) { best = b; bi = i; }
    }
    if (best != SIZE_MAX) {
        const CachedBlock blk = c.blocks[bi];
        c.blocks.erase(c.blocks.begin() + (std::ptrdiff_t)bi);
        c.total -= blk.bytes;
        g_live.push_back(blk);
        return blk.p;
    }
    hipError_t e = hipMallocAsync(&p, want, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        flush_all_caches();
        e = hipMallocAsync(&p, want, st);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw RrError{RR_ENOMEM, "hipMallocAsync(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e)};
    }
    g_live.push_back(CachedBlock{p, want});
    return p;
}

void release_stream_blocks(hipStream_t st) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_caches.size(); ++i) {
        StreamCache& c = g_caches[i];
        if (c.dev != dev || c.st != st) continue;
        for (auto& b : c.blocks) (void)hipFreeAsync(b.p, st);
        g_caches.erase(g_caches.begin() + (std::ptrdiff_t)i);
        return;
    }
}

namespace {
std::mutex g_stream_mu;
std::vector<SideStream> g_free_streams;
}  // namespace

SideStream acquire_side_stream() {
    int dev = 0;
    RR_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_stream_mu);
        for (size_t i = g_free_streams.size(); i-- > 0;)
            if (g_free_streams[i].dev == dev) {
                SideStream s = g_free_streams[i];
                g_free_streams.erase(g_free_streams.begin() + (std::ptrdiff_t)i);
                return s;
            }
    }
    SideStream s;
    s.dev = dev;
    RR_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    RR_HIP(hipEventCreateWithFlags(&s.a, hipEventDisableTiming));
    RR_HIP(hipEventCreateWithFlags(&s.b, hipEventDisableTiming));
    return s;
}

void release_side_stream(const SideStream& s) {
    std::lock_guard<std::mutex> lk(g_stream_mu);
    g_free_streams.push_back(s);
}

void Alloc::put(void* p) const {
    if (!p) return;
    if (custom) {
        a.free(a.ctx, p, (void*)st);
        return;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    size_t bytes = 0;
    for (size_t i = g_live.size(); i-- > 0;)
        if (g_live[i].p == p) {
            bytes = g_live[i].bytes;
            g_live[i] = g_live.back();
            g_live.pop_back();
            break;
        }
    if (bytes == 0) {   // not from Alloc::get: give it straight back
        (void)hipFreeAsync(p, st);
        return;
    }
    StreamCache& c = cache_for(dev, st);
    c.blocks.push_back(CachedBlock{p, bytes});
    c.total += bytes;
    while (c.total > kStreamCacheCap && !c.blocks.empty()) {
        (void)hipFreeAsync(c.blocks.front().p, st);
        c.total -= c.blocks.front().bytes;
        c.blocks.erase(c.blocks.begin());
    }
}

KernelOp kernel_op_of(const rr_precond& P) {
    KernelOp k;
    k.kind = P.op.kind;
    k.n = P.op.n;
    k.d = P.op.d;
    k.pts = P.op.pts;
    k.sqn = P.sqn.as<float>();
    k.xa = P.xa.as<float>();
    k.dm = kernel_record_len(P.op.d);
    k.kconst = P.op.kconst;
    k.scale = P.op.scale;
    k.xd = P.xd.as<double>();
    k.hd = P.hd.as<double>();
    return k;
}

void setup_operator(rr_precond& P, hipStream_t st) {
    const rr_operator& A = P.op;
    const int64_t n = A.n;
    if (is_kernel(A)) {
        const int dm = kernel_record_len(A.d);
        P.sqn.reset(&P.alloc, (size_t)n * sizeof(float));
        launch_sqnorms(A.pts, n, A.d, P.sqn.as<float>(), st);
        P.xa.reset(&P.alloc, (size_t)n * dm * sizeof(float));
        launch_point_records(A.pts, n, A.d, dm, P.xa.as<float>(), st);
        P.xd.reset(&P.alloc, (size_t)n * dm * sizeof(double));
        P.hd.reset(&P.alloc, (size_t)n * sizeof(double));
        launch_point_records64(A.pts, n, A.d, dm, kernel_g64(A.kind, A.kconst), P.xd.as<double>(),
                               P.hd.as<double>(), st);
    } else if (P.opts.prec != RR_PREC_FP64) {
        P.A32.reset(&P.alloc, (size_t)n * n * sizeof(float));
        launch_copy_mat(DT_F64, A.A, A.lda, DT_F32, P.A32.ptr(), n, n, n, st);
    }
}

int operator_part_count(const rr_precond& P) {
    return is_kernel(P.op) ? kernel_matvec_blocks(P.n) : dense_matvec_blocks(P.n);
}

size_t operator_ws_doubles(const rr_precond& P) {
    return is_kernel(P.op) ? kernel_matvec_ws_doubles(P.n, P.op.d, 2) : 0;
}

int apply_operator(const rr_precond& P, const double* u, double mu, double* y, double* dot_part,
                   double* kmv_ws, bool fp64, const int32_t* stop, hipStream_t st) {
    if (is_kernel(P.op)) {
        const KernelOp k = kernel_op_of(P);
        launch_kernel_matvec(k, fp64 || P.opts.prec == RR_PREC_FP64, u, mu, y, dot_part, kmv_ws,
                             stop, st);
        return kernel_matvec_blocks(P.n);
    }
    if (!fp64 && P.A32.ptr())
        launch_dense_matvec(DT_F32, P.n, P.A32.ptr(), P.n, u, mu, y, dot_part, stop, st);
    else
        launch_dense_matvec(DT_F64, P.n, P.op.A, P.op.lda, u, mu, y, dot_part, stop, st);
    return dense_matvec_blocks(P.n);
}

void apply_operator_multi(const rr_precond& P, const double* U, int nr, double mu, double* Y,
                          double* dot_part, double* kmv_ws, bool fp64, hipStream_t st, bool estimate) {
    if (is_kernel(P.op)) {
        const KernelOp k = kernel_op_of(P);
        launch_kernel_matvec_multi(k, fp64 || P.opts.prec == RR_PREC_FP64, U, nr, mu, Y, dot_part,
                                   kmv_ws, nullptr, st, estimate);
        return;
    }
    const int np = operator_part_count(P);
    for (int q = 0; q < nr; ++q)
        apply_operator(P, U + (size_t)q * P.n, mu, Y + (size_t)q * P.n, dot_part + (size_t)q * np,
                       kmv_ws, fp64, nullptr, st);
}

int apply_projected(const rr_precond& P, const double* Kc, const double* r, double rcoef, double* z,
                    double* c_part, double* d, double* rz_part, const int32_t* stop, hipStream_t st) {
    if (P.basisless) {
        // z = rcoef r + Y Kr Y^T r with Y = A_mu Omega (Kc holds Kr^T)
        const KernelOp k = kernel_op_of(P);
        const bool f64 = P.opts.prec == RR_PREC_FP64;
        const double mu = P.per[0].mu;
        launch_kblock_rows(k, f64, P.bl_idx.as<int32_t>(), P.bl_sgn.as<double>(), P.l, r, mu, c_part, stop, st);
        launch_core_apply(P.l, Kc, P.l, c_part, 1, d, stop, st);
        launch_kblock_cols(k, f64, P.bl_idx.as<int32_t>(), P.bl_sgn.as<double>(), P.bl_pos.as<int32_t>(), P.l, d, mu,
                           r, rcoef, z, rz_part, stop, st);
        return kblock_cols_blocks(P.n);
    }
    const int nch = gemv_t_chunks(P.n, P.kb);
    launch_gemv_t(P.n, P.kb, P.Qb.as<double>(), P.n, r, c_part, nch, stop, st);
    launch_core_apply(P.kb, Kc, P.kb, c_part, nch, d, stop, st);
    launch_qd(P.n, P.kb, P.Qb.as<double>(), P.n, d, r, rcoef, z, rz_part, stop, st);
    return qd_blocks(P.n);
}

void apply_projected_pair(const rr_precond& P, const double* K0, const double* K1, const double* R,
                          double rc0, double rc1, double* Z, double* c_part, double* d,
                          double* rz_part, hipStream_t st) {
    const int nch = gemv_t_chunks(P.n, P.kb);
    launch_gemv_t_multi(2, P.n, P.kb, P.Qb.as<double>(), P.n, R, P.n, c_part, nch, nullptr, st);
    launch_core_apply_pair(P.kb, K0, K1, P.kb, c_part, nch, d, nullptr, st);
    launch_qd_multi(2, P.n, P.kb, P.Qb.as<double>(), P.n, d, R, P.n, rc0, rc1, Z, rz_part, nullptr, st);
}

rr_status validate_operator(const rr_operator* A) {
    RR_REQUIRE(A != nullptr, "operator is null");
    RR_REQUIRE(A->n >= 1, "operator n must be >= 1");
    RR_REQUIRE(A->n <= (int64_t)1 << 31, "operator n too large");
    if (A->kind == RR_OP_DENSE) {
        RR_REQUIRE(A->A != nullptr, "dense operator: A is null");
        RR_REQUIRE(A->lda >= A->n, "dense operator: lda < n");
    } else if (A->kind == RR_OP_RBF || A->kind == RR_OP_MATERN32) {
        RR_REQUIRE(A->pts != nullptr, "kernel operator: pts is null");
        RR_REQUIRE(A->d >= 1 && A->d <= 32, "kernel operator: d must be in [1, 32]");
        RR_REQUIRE(std::isfinite(A->kconst) && A->kconst > 0.0, "kernel operator: kconst must be finite and > 0");
        RR_REQUIRE(std::isfinite(A->scale) && A->scale > 0.0, "kernel operator: scale must be finite and > 0");
    } else {
        RR_REQUIRE(false, "unknown operator kind");
    }
    return RR_OK;
}

void require_device() {
    int count = 0;
    const hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        throw RrError{RR_EDEVICE, "no usable HIP device"};
    }
}

}  // namespace rr

rr_precond::~rr_precond() {
    for (rr::Workspace* w : ws_pool) rr_free_workspace(w);
}

void rr_precond_release(rr_precond* P, bool keep_stream) {
    if (!P) return;
    try {
        if (!P->alloc.custom && !keep_stream) {
            P->alloc.st = nullptr;
            for (rr::Workspace* w : P->ws_pool) rr_workspace_null_stream(w);
        }
        delete P;
    } catch (...) {
    }
}

using namespace rr;

extern "C" {

void rr_build_opts_default(rr_build_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->l = 0;
    o->sketch = RR_SK_GAUSSIAN;
    o->seed = 0;
    o->orth = RR_ORTH_SKETCHED_CHOLQR;
    o->prec = RR_PREC_FP64;
    o->tau_rule = RR_TAU_OPT;
    o->rho = 1.0;
    o->power_iters = 4;
    o->power_q = 0;
    o->multi_shift = RR_MULTI_JOINT;
    o->l_max = 0;
    o->ad_factor = 100.0;
    o->basis = RR_BASIS_EXPLICIT;
    o->reorth = 0;
}

void rr_solve_opts_default(rr_solve_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-6;
    o->restart_eta = 1e-2;
    o->maxit = 5000;
    o->check_every = 8;
    o->fp64_ir = -1;
    o->relres_history = nullptr;
    o->history_cap = 0;
    o->use_graph = 0;
    o->certify = 1;
    o->block_kmax = 128;
}

const char* rr_status_string(rr_status s) {
    switch (s) {
        case RR_OK: return "RR_OK";
        case RR_EINVAL: return "RR_EINVAL: invalid argument";
        case RR_ENOMEM: return "RR_ENOMEM: out of device memory or budget";
        case RR_ENOTSPD: return "RR_ENOTSPD: Cholesky failed after the shift ladder";
        case RR_EBREAKDOWN: return "RR_EBREAKDOWN: PCG breakdown";
        case RR_ENOCONV: return "RR_ENOCONV: maximum iterations reached";
        case RR_EDEVICE: return "RR_EDEVICE: HIP device error";
        case RR_EBUSY: return "RR_EBUSY: resource busy";
    }
    return "unknown rr_status";
}

const char* rr_last_error(void) { return g_last_error.c_str(); }

const char* rr_version(void) { return "randrand-gfx950 0.1"; }

void rr_precond_destroy(rr_precond* P) {
    // Every entry point returns only after its device work has completed, so the
    // handle's buffers have no work pending: no device-wide wait here (one would
    // also stall, or break the graph captures of, other threads' streams).  The
    // build and solve streams may be gone by now, so the blocks go to the null
    // stream's cache.
    rr_precond_release(P, false);
}

rr_status rr_precond_shape(const rr_precond* P, int64_t* n, int64_t* l, int32_t* n_mu) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(P != nullptr, "handle is null");
        if (n) *n = P->n;
        if (l) *l = P->l;
        if (n_mu) *n_mu = (int32_t)P->per.size();
        return RR_OK;
    });
}

rr_status rr_precond_export(const rr_precond* P, int32_t mu_index, double* Q_host, double* R_host,
                            double* G_host, double* T_host, double* scalars_host) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(P != nullptr, "handle is null");
        RR_REQUIRE(mu_index >= 0 && mu_index < (int32_t)P->per.size(), "mu_index out of range");
        const PerMu& pm = P->per[mu_index];
        const int64_t n = P->n, l = P->l;
        if (scalars_host) {
            scalars_host[0] = pm.tau;
            scalars_host[1] = pm.normE;
            scalars_host[2] = pm.lam;
            scalars_host[3] = pm.mu;
        }
        if (l == 0) return RR_OK;
        RR_HIP(hipSetDevice(P->device));
        RR_HIP(hipDeviceSynchronize());
        if (Q_host) {
            if (P->basisless) {
                // Q = Y R^{-1} formed on demand (a basis-less handle never stores it)
                Alloc al;
                DBuf Yr(&al, (size_t)n * l * sizeof(double)), Q(&al, (size_t)n * l * sizeof(double));
                DBuf Ri(&al, (size_t)l * l * sizeof(double));
                DBuf ws(&al, ((size_t)4 * l * l + 4 * n) * sizeof(double));
                const KernelOp k = kernel_op_of(*P);
                launch_kblock_y(k, P->opts.prec == RR_PREC_FP64, P->bl_idx.as<int32_t>(), P->bl_sgn.as<double>(), l,
                                pm.mu, 0, n, nullptr, nullptr, Yr.as<double>(), l, nullptr);
                launch_tri_inv_upper(pm.R.as<double>(), l, l, Ri.as<double>(), l, nullptr);
                // Yr (row-major n x l) is the column-major l x n matrix Y^T
                launch_gemm(DT_F64, true, DT_F64, false, n, l, l, Yr.ptr(), l, Ri.ptr(), l, Q.as<double>(), n, 1.0,
                            0.0, ws.as<double>(), (size_t)4 * l * l + 4 * n, nullptr);
                RR_HIP(hipDeviceSynchronize());
                RR_HIP(hipMemcpy(Q_host, Q.ptr(), (size_t)n * l * sizeof(double), hipMemcpyDeviceToHost));
            } else if (!P->joint) {
                RR_HIP(hipMemcpy(Q_host, P->Qb.ptr(), (size_t)n * l * sizeof(double), hipMemcpyDeviceToHost));
            } else {
                Alloc al;
                DBuf Q(&al, (size_t)n * l * sizeof(double));
                DBuf ws(&al, gemm_ws_doubles(n, l, P->kb) * sizeof(double));
                launch_gemm(DT_F64, false, DT_F64, false, n, l, P->kb, P->Qb.ptr(), n, pm.Qred.ptr(),
                            P->kb, Q.as<double>(), n, 1.0, 0.0, ws.as<double>(),
                            gemm_ws_doubles(n, l, P->kb), nullptr);
                RR_HIP(hipDeviceSynchronize());
                RR_HIP(hipMemcpy(Q_host, Q.ptr(), (size_t)n * l * sizeof(double), hipMemcpyDeviceToHost));
            }
        }
        const size_t ll = (size_t)l * l * sizeof(double);
        if (R_host) RR_HIP(hipMemcpy(R_host, pm.R.ptr(), ll, hipMemcpyDeviceToHost));
        if (G_host) RR_HIP(hipMemcpy(G_host, pm.G.ptr(), ll, hipMemcpyDeviceToHost));
        if (T_host) RR_HIP(hipMemcpy(T_host, pm.T.ptr(), ll, hipMemcpyDeviceToHost));
        return RR_OK;
    });
}

rr_status rr_precond_export_omega(const rr_precond* P, double* Omega_host) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(P != nullptr && Omega_host != nullptr, "null argument");
        if (P->l == 0) return RR_OK;
        RR_HIP(hipSetDevice(P->device));
        Alloc al;
        DBuf O(&al, (size_t)P->n * P->l * sizeof(double));
        if (P->basisless)
            launch_colsample_fill(DT_F64, P->n, P->l, P->n, P->bl_idx.as<int32_t>(), P->bl_sgn.as<double>(), O.ptr(),
                                  nullptr);
        else
            launch_copy_mat(P->omega_dt, P->Omega.ptr(), P->n, DT_F64, O.ptr(), P->n, P->n, P->l, nullptr);
        RR_HIP(hipDeviceSynchronize());
        RR_HIP(hipMemcpy(Omega_host, O.ptr(), (size_t)P->n * P->l * sizeof(double), hipMemcpyDeviceToHost));
        return RR_OK;
    });
}

rr_status rr_kernel_to_dense(const rr_operator* kop, void* A_out, int32_t dtype, int64_t lda,
                             void* hip_stream) {
    return guarded([&]() -> rr_status {
        validate_operator(kop);
        RR_REQUIRE(is_kernel(*kop), "rr_kernel_to_dense needs a kernel operator");
        RR_REQUIRE(A_out != nullptr, "A_out is null");
        RR_REQUIRE(lda >= kop->n, "lda < n");
        RR_REQUIRE(dtype >= 0 && dtype <= 2, "dtype must be 0 (f64), 1 (f32) or 2 (bf16)");
        require_device();
        KernelOp k;
        k.kind = kop->kind; k.n = kop->n; k.d = kop->d; k.pts = kop->pts; k.sqn = nullptr;
        k.xa = nullptr; k.dm = 0;
        k.kconst = kop->kconst; k.scale = kop->scale;
        hipStream_t st = (hipStream_t)hip_stream;
        launch_kernel_to_dense(k, A_out, dtype, lda, st);
        RR_HIP(hipGetLastError());
        RR_HIP(hipStreamSynchronize(st));
        return RR_OK;
    });
}

rr_status rr_apply_operator_block(const rr_operator* A, double mu, int32_t prec, const double* U,
                                 int32_t nr, double* Y, void* hip_stream) {
    return guarded([&]() -> rr_status {
        validate_operator(A);
        RR_REQUIRE(U != nullptr && Y != nullptr, "U or Y is null");
        RR_REQUIRE(nr >= 1 && nr <= 4096, "nr must be in [1, 4096]");
        RR_REQUIRE(std::isfinite(mu), "mu must be finite");
        RR_REQUIRE(prec >= 0 && prec <= 2, "unknown precision");
        require_device();
        hipStream_t st = (hipStream_t)hip_stream;
        rr_precond P;   // a transient handle holding only the operator view
        P.op = *A;
        P.n = A->n;
        P.opts.prec = prec;
        P.alloc.st = st;
        const size_t ws = is_kernel(*A) ? kernel_matvec_ws_doubles(A->n, A->d, nr) : 0;
        DBuf part(&P.alloc, ((size_t)operator_part_count(P) * nr + 1) * sizeof(double));
        DBuf kws(&P.alloc, (ws + 1) * sizeof(double));
        setup_operator(P, st);
        apply_operator_multi(P, U, nr, mu, Y, part.as<double>(), kws.as<double>(),
                             prec == RR_PREC_FP64, st);
        RR_HIP(hipGetLastError());
        RR_HIP(hipStreamSynchronize(st));
        return RR_OK;
    });
}

rr_status rr_operator_delta_norm(const rr_operator* A, int32_t prec, int32_t iters, uint64_t seed,
                                 double* out_host, void* hip_stream) {
    return guarded([&]() -> rr_status {
        validate_operator(A);
        RR_REQUIRE(out_host != nullptr, "out is null");
        RR_REQUIRE(prec >= 0 && prec <= 2, "unknown precision");
        RR_REQUIRE(iters >= 1 && iters <= 1000, "iters must be in [1, 1000]");
        require_device();
        hipStream_t st = (hipStream_t)hip_stream;
        rr_precond P;
        P.op = *A;
        P.n = A->n;
        P.opts.prec = prec;
        P.alloc.st = st;
        const int64_t n = A->n;
        if (prec == RR_PREC_FP64) {
            *out_host = 0.0;   // the working operator is the float64 one
            return RR_OK;
        }
        const size_t ws = is_kernel(*A) ? kernel_matvec_ws_doubles(n, A->d, 1) : 0;
        DBuf part(&P.alloc, ((size_t)operator_part_count(P) + 1) * sizeof(double));
        DBuf kws(&P.alloc, (ws + 1) * sizeof(double));
        DBuf v(&P.alloc, n * sizeof(double)), y1(&P.alloc, n * sizeof(double)), y2(&P.alloc, n * sizeof(double));
        DBuf vp(&P.alloc, ((size_t)vec_blocks(n) + 1) * sizeof(double)), sc(&P.alloc, 4 * sizeof(double));
        setup_operator(P, st);
        launch_gauss_fill(v.ptr(), DT_F64, n, 1, n, seed, st);
        launch_dot_part(n, v.as<double>(), v.as<double>(), vp.as<double>(), st);
        launch_normalize(n, v.as<double>(), v.as<double>(), vp.as<double>(), vec_blocks(n), sc.as<double>() + 1, st);
        for (int it = 0; it < iters; ++it) {
            apply_operator(P, v.as<double>(), 0.0, y1.as<double>(), part.as<double>(), kws.as<double>(), false,
                           nullptr, st);
            apply_operator(P, v.as<double>(), 0.0, y2.as<double>(), part.as<double>(), kws.as<double>(), true,
                           nullptr, st);
            launch_axpby_mat(1.0, y1.as<double>(), n, -1.0, y2.as<double>(), n, y1.as<double>(), n, n, 1, st);
            launch_dot_part(n, y1.as<double>(), y1.as<double>(), vp.as<double>(), st);
            launch_normalize(n, v.as<double>(), y1.as<double>(), vp.as<double>(), vec_blocks(n), sc.as<double>(), st);
        }
        RR_HIP(hipGetLastError());
        RR_HIP(hipMemcpyAsync(out_host, sc.ptr(), sizeof(double), hipMemcpyDeviceToHost, st));
        RR_HIP(hipStreamSynchronize(st));
        return RR_OK;
    });
}

rr_status rr_apply_operator(const rr_operator* A, double mu, int32_t prec, const double* u, double* y,
                            void* hip_stream) {
    return rr_apply_operator_block(A, mu, prec, u, 1, y, hip_stream);
}

rr_status rr_random_matrix(int32_t kind, uint64_t seed, int64_t rows, int64_t cols, double* out,
                           void* hip_stream) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(out != nullptr, "out is null");
        RR_REQUIRE(rows >= 1 && cols >= 1, "rows and cols must be >= 1");
        RR_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (Gaussian) or 1 (SRHT)");
        require_device();
        hipStream_t st = (hipStream_t)hip_stream;
        if (kind == 0) {
            launch_gauss_fill(out, DT_F64, rows, cols, rows, seed, st);
        } else {
            int64_t s = 1;
            while (s < rows) s *= 2;
            RR_REQUIRE(cols <= s, "SRHT: cols exceeds padded size");
            Alloc al;
            al.st = st;
            DBuf perm(&al, (size_t)s * sizeof(int32_t));
            DBuf srows(&al, (size_t)cols * sizeof(int32_t));
            DBuf D(&al, (size_t)rows * sizeof(float));
            launch_srht_prepare(rows, cols, seed, s, perm.as<int32_t>(), srows.as<int32_t>(), D.as<float>(), st);
            launch_srht_fill(out, DT_F64, rows, cols, rows, D.as<float>(), srows.as<int32_t>(), st);
            RR_HIP(hipStreamSynchronize(st));
        }
        RR_HIP(hipGetLastError());
        RR_HIP(hipStreamSynchronize(st));
        return RR_OK;
    });
}

rr_status rr_theta_apply(uint64_t seed, int64_t n, int64_t k, const double* Y, double* S, void* hip_stream) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(Y != nullptr && S != nullptr, "Y or S is null");
        RR_REQUIRE(n >= 1 && k >= 1, "n and k must be >= 1");
        require_device();
        hipStream_t st = (hipStream_t)hip_stream;
        Alloc al;
        al.st = st;
        DBuf Yt(&al, (size_t)n * k * sizeof(double));
        launch_transpose_f64(DT_F64, n, k, Y, n, Yt.as<double>(), k, st);
        launch_theta_apply(n, k, seed + 1, Yt.as<double>(), k, S, 2 * k, st);
        RR_HIP(hipGetLastError());
        return RR_OK;
    });
}

}  // extern "C"
