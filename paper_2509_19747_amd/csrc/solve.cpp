// rr_solve: C-RandRAND PCG with restarts (Algorithm RandRAND_PCG steps 5-11,
// Section 6.2; restart after every residual drop by eta, Section 7 setup).
//
// One iteration (Hestenes-Stiefel order):
//   w = A_mu p, p^T w        (operator kernel, fused dot partials)
//   alpha = rho / p^T w       (one-block scalar kernel)
//   x += alpha p; r -= alpha w; ||r||^2
//   stop test on ||r|| (device flag: every later kernel of the batch is a no-op)
//   z = r + Q (K (Q^T r)), r^T z   (eq. g_randrand_explicit with the refined
//                                   projector folded into K)
//   beta = r^T z / rho; p = z + beta p
// The host launches `check_every` iterations at a time (optionally as one
// replayed hipGraph) and reads the 8-byte state once per batch.  At every
// restart the residual is recomputed from x, with the float64 operator when
// outer iterative refinement is on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.hpp"

using namespace rr;

namespace rr {

struct Workspace {
    Alloc al;
    int64_t n = 0, kb = 0;
    DBuf r, p, z, w;
    DBuf op_part, rr_part, rz_part, c_part, d, kws, state, flag, scal, hist;
    int32_t hist_cap = 0;
    int op_parts = 0, nch = 0;
    PooledStream cap;            // private stream used for graph capture/replay
};

static Workspace* make_workspace(const rr_precond& P, int32_t maxit, hipStream_t st) {
    Workspace* W = new Workspace();
    W->al = P.alloc;
    if (!W->al.custom) W->al.st = st;   // ordered with the solve that first uses it
    W->n = P.n;
    W->kb = P.kb;
    const int64_t n = P.n;
    const Alloc* al = &W->al;
    W->r.reset(al, n * sizeof(double));
    W->p.reset(al, n * sizeof(double));
    W->z.reset(al, n * sizeof(double));
    W->w.reset(al, n * sizeof(double));
    W->op_parts = operator_part_count(P);
    W->op_part.reset(al, (size_t)std::max(W->op_parts, 1) * sizeof(double));
    W->rr_part.reset(al, (size_t)vec_blocks(n) * sizeof(double));
    W->rz_part.reset(al, (size_t)std::max(qd_blocks(n), vec_blocks(n)) * sizeof(double));
    W->nch = P.kb > 0 ? gemv_t_chunks(n, P.kb) : 1;
    W->c_part.reset(al, (size_t)W->nch * std::max<int64_t>(P.kb, 1) * sizeof(double));
    W->d.reset(al, (size_t)std::max<int64_t>(P.kb, 1) * sizeof(double));
    W->kws.reset(al, (operator_ws_doubles(P) + 1) * sizeof(double));
    W->state.reset(al, sizeof(CgState));
    W->flag.reset(al, 16);
    W->scal.reset(al, 16 * sizeof(double));
    W->hist_cap = maxit + 2;
    W->hist.reset(al, (size_t)W->hist_cap * sizeof(double));
    return W;
}

}  // namespace rr

void rr_free_workspace(rr::Workspace* w) { delete w; }
void rr_workspace_null_stream(rr::Workspace* w) {
    if (w && !w->al.custom) w->al.st = nullptr;
}

namespace {

struct Solver {
    const rr_precond& P;
    Workspace& W;
    hipStream_t st;
    double mu;
    const double* Kc;

    void sync() { RR_HIP(hipStreamSynchronize(st)); }

    // z = P r with partials of r^T z in W.rz_part; returns the partial count.
    int precond(const double* r, double* z, const int32_t* stop) {
        if (P.l == 0) {
            launch_copy_vec(P.n, r, z, st);   // only used outside the iteration
            launch_dot_part(P.n, r, z, W.rz_part.as<double>(), st);
            return vec_blocks(P.n);
        }
        return apply_projected(P, Kc, r, 1.0, z, W.c_part.as<double>(), W.d.as<double>(),
                               W.rz_part.as<double>(), stop, st);
    }

    // r = b - A x (float64 operator if fp64); returns ||r||^2 on the host.
    double true_residual(const double* b, const double* x, bool fp64) {
        apply_operator(P, x, mu, W.w.as<double>(), W.op_part.as<double>(), W.kws.as<double>(), fp64,
                       nullptr, st);
        launch_residual(P.n, b, W.w.as<double>(), W.r.as<double>(), W.rr_part.as<double>(), st);
        launch_scal_set(W.rr_part.as<double>(), vec_blocks(P.n), W.scal.as<double>(), st);
        RR_HIP(hipGetLastError());
        double rr2 = 0.0;
        RR_HIP(hipMemcpyAsync(&rr2, W.scal.ptr(), sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        return rr2;
    }

    // One PCG iteration, all on the device.
    void iteration(double* x) {
        CgState* s = W.state.as<CgState>();
        const int32_t* stop = &s->stop;
        const int64_t n = P.n;
        double* p = W.p.as<double>();
        double* r = W.r.as<double>();
        double* w = W.w.as<double>();
        const int np = apply_operator(P, p, mu, w, W.op_part.as<double>(), W.kws.as<double>(), false,
                                      stop, st);
        launch_scal_alpha(W.op_part.as<double>(), np, s, st);
        launch_xr_update(n, x, r, p, w, s, W.rr_part.as<double>(), st);
        launch_scal_rr(W.rr_part.as<double>(), vec_blocks(n), s, st);
        if (P.l > 0) {
            const int nz = apply_projected(P, Kc, r, 1.0, W.z.as<double>(), W.c_part.as<double>(),
                                           W.d.as<double>(), W.rz_part.as<double>(), stop, st);
            launch_scal_beta(W.rz_part.as<double>(), nz, s, st);
            launch_p_update(n, W.z.as<double>(), p, s, st);
        } else {
            launch_scal_beta(W.rr_part.as<double>(), vec_blocks(n), s, st);
            launch_p_update(n, r, p, s, st);
        }
    }
};

}  // namespace

static rr_status validate_solve(const rr_precond* P, const rr_solve_opts& o) {
    RR_REQUIRE(P != nullptr, "handle is null");
    RR_REQUIRE(std::isfinite(o.tol) && o.tol > 0.0 && o.tol < 1.0, "tol must be in (0, 1)");
    RR_REQUIRE(std::isfinite(o.restart_eta) && o.restart_eta > 0.0 && o.restart_eta < 1.0,
               "restart_eta must be in (0, 1)");
    RR_REQUIRE(o.maxit >= 1 && o.maxit <= 100000000, "maxit must be >= 1");
    RR_REQUIRE(o.check_every >= 1 && o.check_every <= 4096, "check_every must be in [1, 4096]");
    RR_REQUIRE(o.history_cap >= 0, "history_cap must be >= 0");
    RR_REQUIRE(o.history_cap == 0 || o.relres_history != nullptr, "relres_history is null");
    RR_REQUIRE(o.method >= RR_METHOD_C && o.method <= RR_METHOD_SPLIT_R, "unknown method");
    RR_REQUIRE(o.krylov >= RR_KRYLOV_CG && o.krylov <= RR_KRYLOV_BLOCK_CG, "unknown Krylov method");
    RR_REQUIRE(o.block_kmax >= 1 && o.block_kmax <= 4096, "block_kmax must be in [1, 4096]");
    return RR_OK;
}

rr_status rr_solve_general(const rr_precond* Pc, int32_t mu_index, const double* b, double* x,
                           const rr_solve_opts& o, rr_solve_info* info, hipStream_t st);

extern "C" rr_status rr_solve(const rr_precond* Pc, int32_t mu_index, const double* b, double* x,
                              const rr_solve_opts* opts_in, rr_solve_info* info, void* hip_stream) {
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->status = RR_EINVAL;
    }
    rr_solve_opts o;
    if (opts_in) o = *opts_in; else rr_solve_opts_default(&o);
    rr_status rs = guarded([&]() -> rr_status {
        validate_solve(Pc, o);
        RR_REQUIRE(mu_index >= 0 && mu_index < (int32_t)Pc->per.size(), "mu_index out of range");
        RR_REQUIRE(b != nullptr && x != nullptr, "b or x is null");
        RR_REQUIRE(o.krylov == RR_KRYLOV_CG || o.krylov == RR_KRYLOV_MINRES,
                   "rr_solve runs CG or MINRES (block methods: rr_solve_batch)");
        require_device();
        rr_precond& P = const_cast<rr_precond&>(*Pc);
        hipStream_t st = (hipStream_t)hip_stream;
        if (o.method != RR_METHOD_C || o.krylov != RR_KRYLOV_CG)
            return rr_solve_general(Pc, mu_index, b, x, o, info, st);
        // a workspace of this handle's pool (a new one if every pooled one is busy
        // or too small); returned to the pool when the solve ends
        Workspace* wsp = nullptr;
        {
            std::lock_guard<std::mutex> lock(P.ws_mu);
            for (size_t i = P.ws_pool.size(); i-- > 0;)
                if (P.ws_pool[i]->hist_cap >= o.maxit + 2) {
                    wsp = P.ws_pool[i];
                    P.ws_pool.erase(P.ws_pool.begin() + (std::ptrdiff_t)i);
                    break;
                }
        }
        if (!wsp) wsp = make_workspace(P, o.maxit, st);
        struct WsReturn {
            rr_precond& P;
            Workspace* w;
            ~WsReturn() {
                std::lock_guard<std::mutex> lock(P.ws_mu);
                P.ws_pool.push_back(w);
            }
        } ws_return{P, wsp};
        Workspace& W = *wsp;
        const PerMu& pm = P.per[mu_index];
        Solver S{P, W, st, pm.mu, P.l > 0 ? pm.Kc.as<double>() : nullptr};
        const int64_t n = P.n;
        // outer float64 refinement: by default whenever the working operator is not the
        // float64 one (the residual at every restart then uses the float64 operator)
        const bool ir = (o.fp64_ir == 1) || (o.fp64_ir == -1 && P.opts.prec != RR_PREC_FP64);

        // NaN/Inf scan of b (and x0) before any arithmetic
        // (and whether x0 is zero: then the first residual is b itself, no operator product)
        RR_HIP(hipMemsetAsync(W.flag.ptr(), 0, 2 * sizeof(int32_t), st));
        launch_nonfinite(n, b, W.flag.as<int32_t>(), st);
        launch_nonfinite(n, x, W.flag.as<int32_t>(), st, W.flag.as<int32_t>() + 1);
        int32_t flags[2] = {0, 0};
        RR_HIP(hipMemcpyAsync(flags, W.flag.ptr(), 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        S.sync();
        RR_REQUIRE(flags[0] == 0, "b or x0 contains NaN or Inf");
        const bool x0_zero = flags[1] == 0;

        const double t0 = now_ms();
        launch_dot_part(n, b, b, W.rr_part.as<double>(), st);
        launch_scal_set(W.rr_part.as<double>(), vec_blocks(n), W.scal.as<double>(), st);
        double bb = 0.0;
        RR_HIP(hipMemcpyAsync(&bb, W.scal.ptr(), sizeof(double), hipMemcpyDeviceToHost, st));
        S.sync();
        const double nb = std::sqrt(bb);
        rr_solve_info inf{};
        inf.tau = pm.tau; inf.normE = pm.normE; inf.lamhat = pm.lam; inf.orth_err = P.orth_err;
        inf.ms_build = P.ms_build;
        std::vector<double> hist;
        if (nb == 0.0) {
            RR_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
            S.sync();
            inf.status = RR_OK;
            inf.ms_solve = now_ms() - t0;
            if (info) *info = inf;
            return RR_OK;
        }

        hipGraphExec_t gexec = nullptr;
        hipGraph_t graph = nullptr;
        struct GraphGuard {
            hipGraphExec_t* e; hipGraph_t* g;
            ~GraphGuard() { if (*e) (void)hipGraphExecDestroy(*e); if (*g) (void)hipGraphDestroy(*g); }
        } gg{&gexec, &graph};

        bool graph_failed = false;
        int its = 0, cycles = 0;
        rr_status result = RR_ENOCONV;
        double relres = 1.0;
        while (true) {
            double rn = nb;
            if (x0_zero && cycles == 0) launch_copy_vec(n, b, W.r.as<double>(), st);   // r0 = b - A 0
            else rn = std::sqrt(S.true_residual(b, x, ir));
            relres = rn / nb;
            if (its < o.history_cap) o.relres_history[its] = relres;
            if (!std::isfinite(rn)) { result = RR_EBREAKDOWN; break; }
            if (rn <= o.tol * nb) { result = RR_OK; break; }
            if (its >= o.maxit) { result = RR_ENOCONV; break; }
            ++cycles;
            const double target = std::max(o.restart_eta * rn, o.tol * nb);
            const int nz = S.precond(W.r.as<double>(), W.z.as<double>(), nullptr);
            launch_state_init(W.state.as<CgState>(), W.rz_part.as<double>(), nz, target * target,
                              o.maxit, its, W.hist.as<double>(), W.hist_cap, st);
            launch_copy_vec(n, W.z.as<double>(), W.p.as<double>(), st);
            RR_HIP(hipGetLastError());
            CgState hs{};
            while (true) {
                if (o.use_graph && !graph_failed) {
                    // capture on a private non-default stream; the caller's stream
                    // has been synchronised, so ordering is preserved
                    hipStream_t cst = W.cap.get();
                    S.sync();
                    if (!gexec) {
                        Solver C{P, W, cst, S.mu, S.Kc};
                        // relaxed: the capture holds kernel launches only, and allocation or copy calls
                        // of other threads (a server's other requests) must not invalidate it
                        RR_HIP(hipStreamBeginCapture(cst, hipStreamCaptureModeRelaxed));
                        for (int k = 0; k < o.check_every; ++k) C.iteration(x);
                        if (hipStreamEndCapture(cst, &graph) != hipSuccess) {
                            // an invalidated capture ran nothing: the solve continues with
                            // eager launches of the same kernels, and info.graph_fallbacks
                            // reports it
                            (void)hipGetLastError();
                            if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
                            graph_failed = true;
                            continue;
                        }
                        RR_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
                    }
                    RR_HIP(hipGraphLaunch(gexec, cst));
                    RR_HIP(hipStreamSynchronize(cst));
                } else {
                    for (int k = 0; k < o.check_every; ++k) S.iteration(x);
                }
                RR_HIP(hipGetLastError());
                RR_HIP(hipMemcpyAsync(&hs, W.state.ptr(), sizeof(CgState), hipMemcpyDeviceToHost, st));
                S.sync();
                if (hs.stop != STOP_NONE) break;
            }
            // copy the per-iteration ||r||^2 of this cycle into the host history
            if (o.history_cap > 0 && hs.iters > its) {
                const int a = its + 1, e = std::min(hs.iters, o.history_cap - 1);
                if (e >= a) {
                    hist.resize((size_t)(e - a + 1));
                    RR_HIP(hipMemcpy(hist.data(), W.hist.as<double>() + a, hist.size() * sizeof(double),
                                     hipMemcpyDeviceToHost));
                    for (int q = a; q <= e; ++q) o.relres_history[q] = std::sqrt(hist[q - a]) / nb;
                }
            }
            its = hs.iters;
            if (hs.stop == STOP_BREAKDOWN) { result = RR_EBREAKDOWN; relres = std::sqrt(hs.rr) / nb; break; }
            // STOP_TARGET or STOP_MAXIT: recompute the true residual (restart)
        }
        inf.iters = its;
        inf.graph_fallbacks = graph_failed ? 1 : 0;
        inf.restarts = std::max(cycles - 1, 0);
        inf.relres_work = relres;
        inf.ms_solve = now_ms() - t0;
        inf.relres_fp64 = std::nan("");
        if (ir || P.opts.prec == RR_PREC_FP64) {
            // the last true residual already came from the float64 operator
            inf.relres_fp64 = relres;
        } else if (o.certify) {
            const double rf = std::sqrt(S.true_residual(b, x, true));
            inf.relres_fp64 = rf / nb;
        }
        inf.status = result;
        if (info) *info = inf;
        if (result != RR_OK) {
            set_error(result == RR_ENOCONV ? "maximum iterations reached" : "PCG breakdown (p^T A p <= 0 or r^T z <= 0)");
        }
        return result;
    });
    if (info && rs != RR_OK && info->status == RR_EINVAL && rs != RR_EINVAL) info->status = rs;
    if (info && rs == RR_EINVAL) info->status = RR_EINVAL;
    return rs;
}

// Several right-hand sides: one independent PCG recurrence per column.
extern "C" rr_status rr_solve_batch(const rr_precond* P, const int32_t* mu_index_per_col,
                                    const double* B, int64_t ldb, int32_t nrhs, double* X,
                                    int64_t ldx, const rr_solve_opts* opts, rr_solve_info* infos,
                                    void* hip_stream) {
    return rr::solve_batch_with(P, mu_index_per_col, B, ldb, nrhs, X, ldx, opts, infos, hip_stream, nullptr);
}

rr_status rr::solve_batch_with(const rr_precond* P, const int32_t* mu_index_per_col, const double* B,
                               int64_t ldb, int32_t nrhs, double* X, int64_t ldx, const rr_solve_opts* opts,
                               rr_solve_info* infos, void* hip_stream, BatchRunner* runner) {
    rr_solve_opts o;
    if (opts) o = *opts; else rr_solve_opts_default(&o);
    rr_status v = guarded([&]() -> rr_status {
        validate_solve(P, o);
        RR_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        RR_REQUIRE(mu_index_per_col != nullptr, "mu_index_per_col is null");
        RR_REQUIRE(B != nullptr && X != nullptr, "B or X is null");
        RR_REQUIRE(ldb >= P->n && ldx >= P->n, "ldb and ldx must be >= n");
        for (int j = 0; j < nrhs; ++j)
            RR_REQUIRE(mu_index_per_col[j] >= 0 && mu_index_per_col[j] < (int32_t)P->per.size(),
                       "mu index out of range");
        RR_REQUIRE(o.history_cap == 0, "relres_history is not supported for batched solves");
        RR_REQUIRE(o.method == RR_METHOD_C && o.krylov != RR_KRYLOV_MINRES,
                   "batched solves run C-RandRAND with CG, BLOCK_MINRES or BLOCK_CG");
        RR_REQUIRE(!P->basisless, "batched solves need an explicit basis");
        return RR_OK;
    });
    if (v != RR_OK) return v;
    if (o.krylov == RR_KRYLOV_BLOCK_MINRES || o.krylov == RR_KRYLOV_BLOCK_CG)
        return rr_solve_block(P, mu_index_per_col, B, ldb, nrhs, X, ldx, &o, infos, hip_stream);
    return rr_solve_batch_fused(P, mu_index_per_col, B, ldb, nrhs, X, ldx, &o, infos, hip_stream, runner);
}
