// rr_solve_batch: m independent C-RandRAND PCG recurrences (one per column, each
// with its own shift from the handle) advanced together.
//
// Per iteration, for all columns at once:
//   W = A_mu P      one operator product for all columns (kernel operators: the
//                   float32 kernel entries widened to float64 on FP64 MFMA)
//   alpha_j, x_j, r_j, ||r_j||^2, per-column stop test (column run flags)
//   Z = R + Qb (Kc_{mu(j)} (Qb^T R))   (GEMMs over the joint basis, Section 5.1)
//   beta_j, p_j
// Restarts follow the single solve exactly per column (Algorithm RandRAND_PCG
// step 10 with eta): a column that reaches its cycle target stops; at the next
// host check its true residual b_j - A_mu x_j is recomputed and it either finishes
// or starts a new cycle.  Columns that have stopped are not updated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

using namespace rr;

rr_status rr_solve_batch_fused(const rr_precond* Pc, const int32_t* mu_index_per_col,
                               const double* B, int64_t ldb, int32_t nrhs, double* X, int64_t ldx,
                               const rr_solve_opts* o, rr_solve_info* infos, void* hip_stream,
                               rr::BatchRunner* runner) {
    if (infos)
        for (int j = 0; j < nrhs; ++j) { std::memset(&infos[j], 0, sizeof(rr_solve_info)); infos[j].status = RR_EINVAL; }
    return guarded([&]() -> rr_status {
        require_device();
        const rr_precond& P = *Pc;
        hipStream_t st = (hipStream_t)hip_stream;
        const int64_t n = P.n, m = nrhs;
        const double t0 = now_ms();
        Batch Bt(P, st, m, runner != nullptr);
        // per-column shifts and the set of shifts in use
        std::vector<double> hmu(m);
        std::vector<int> used(P.per.size(), 0);
        for (int64_t j = 0; j < m; ++j) { hmu[j] = P.per[mu_index_per_col[j]].mu; used[mu_index_per_col[j]] = 1; }
        for (size_t g = 0; g < used.size(); ++g) if (used[g]) Bt.mus_used.push_back((int)g);
        Bt.setup_single_shift();
        // iteration batches in the serving loop's grouped replays when the column block
        // has their shape (one shift, the MFMA kernel product, streaming projection)
        const bool grouped = runner != nullptr && Bt.group_ok();
        RR_HIP(hipMemcpyAsync(Bt.mucol.ptr(), hmu.data(), m * sizeof(double), hipMemcpyHostToDevice, st));
        RR_HIP(hipMemcpyAsync(Bt.muidx.ptr(), mu_index_per_col, m * sizeof(int32_t), hipMemcpyHostToDevice, st));

        // NaN / Inf scan
        // (and whether X0 is zero: then the first residuals are the columns of B)
        bool x0_zero = false;
        {
            DBuf flag(Bt.al, 16);
            RR_HIP(hipMemsetAsync(flag.ptr(), 0, 2 * sizeof(int32_t), st));
            for (int64_t j = 0; j < m; ++j) {
                launch_nonfinite(n, B + j * ldb, flag.as<int32_t>(), st);
                launch_nonfinite(n, X + j * ldx, flag.as<int32_t>(), st, flag.as<int32_t>() + 1);
            }
            int32_t flags[2] = {0, 0};
            RR_HIP(hipMemcpyAsync(flags, flag.ptr(), 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            RR_HIP(hipStreamSynchronize(st));
            RR_REQUIRE(flags[0] == 0, "B or X0 contains NaN or Inf");
            x0_zero = flags[1] == 0;
        }
        const bool ir = (o->fp64_ir == 1) || (o->fp64_ir == -1 && P.opts.prec != RR_PREC_FP64);
        const std::vector<double> bb = Bt.coldots(B, ldb, B, ldb);
        std::vector<double> nb(m);
        for (int64_t j = 0; j < m; ++j) nb[j] = std::sqrt(bb[j]);

        std::vector<int> done(m, 0), cycles(m, 0), status(m, RR_ENOCONV), iters(m, 0);
        std::vector<double> relres(m, 1.0);
        std::vector<int32_t> hstart(m, 0);
        std::vector<double> htarget(m, 0.0);
        std::vector<BState> hs(m);
        std::vector<int> pending(m, 1);   // needs a true-residual check
        double* Xd = X;

        bool first_pass = true;
        auto restart_pass = [&]() {
            // T = B - A_mu X for every column (T = B for a zero X0); decide per pending column
            std::vector<double> rr;
            if (first_pass && x0_zero) {
                launch_copy_mat(DT_F64, B, ldb, DT_F64, Bt.T.as<double>(), n, n, m, st);
                rr = bb;
            } else {
                // the true residuals of the columns checked now (those still running
                // or finished keep their state; their columns of T are not used)
                std::vector<int32_t> cols;
                for (int64_t j = 0; j < m; ++j)
                    if (pending[j] && !done[j]) cols.push_back((int32_t)j);
                Bt.product_cols(Xd, ldx, Bt.T.as<double>(), ir, cols, hmu);
                launch_bresid(n, m, B, ldb, Bt.T.as<double>(), Bt.T.as<double>(), st);
                rr = Bt.coldots(Bt.T.as<double>(), n, Bt.T.as<double>(), n);
            }
            first_pass = false;
            bool any = false;
            for (int64_t j = 0; j < m; ++j) {
                hstart[j] = 0;
                if (!pending[j] || done[j]) continue;
                pending[j] = 0;
                const double rn = std::sqrt(rr[j]);
                relres[j] = nb[j] > 0.0 ? rn / nb[j] : 0.0;
                if (nb[j] == 0.0 || rn <= o->tol * nb[j]) { done[j] = 1; status[j] = RR_OK; continue; }
                if (!std::isfinite(rn)) { done[j] = 1; status[j] = RR_EBREAKDOWN; continue; }
                if (iters[j] >= o->maxit) { done[j] = 1; status[j] = RR_ENOCONV; continue; }
                ++cycles[j];
                const double target = std::max(o->restart_eta * rn, o->tol * nb[j]);
                htarget[j] = target * target;
                hstart[j] = 1;
                any = true;
            }
            if (!any) return false;
            RR_HIP(hipMemcpyAsync(Bt.start.ptr(), hstart.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, st));
            RR_HIP(hipMemcpyAsync(Bt.target2.ptr(), htarget.data(), m * sizeof(double), hipMemcpyHostToDevice, st));
            // new cycle for the started columns: r = T, z = P r, rho = r^T z, p = z
            launch_copy_flagged(n, m, Bt.T.as<double>(), n, Bt.R.as<double>(), n, Bt.start.as<int32_t>(), st);
            Bt.precond(Bt.T.as<double>(), Bt.Z.as<double>());
            launch_coldot(n, m, Bt.T.as<double>(), n, Bt.Z.as<double>(), n, Bt.parts.as<double>(), st);
            launch_bstate_start(ColParts{Bt.parts.as<double>(), Bt.nch, m, 1}, m, Bt.state.as<BState>(),
                                Bt.start.as<int32_t>(),
                                Bt.target2.as<double>(), o->maxit, st);
            launch_copy_flagged(n, m, Bt.Z.as<double>(), n, Bt.Pm.as<double>(), n, Bt.start.as<int32_t>(), st);
            RR_HIP(hipGetLastError());
            return true;
        };

        // iteration counters live in the device state; seed them
        for (int64_t j = 0; j < m; ++j) { hs[j] = BState{}; hs[j].iters = 0; }
        RR_HIP(hipMemcpyAsync(Bt.state.ptr(), hs.data(), m * sizeof(BState), hipMemcpyHostToDevice, st));
        // optional hipGraph of one batch of check_every iterations, captured on a
        // private stream the first time and replayed after every host check
        PooledStream capture;
        hipStream_t cap = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        struct GraphGuard {
            hipGraph_t* g; hipGraphExec_t* e;
            ~GraphGuard() {
                if (*e) (void)hipGraphExecDestroy(*e);
                if (*g) (void)hipGraphDestroy(*g);
            }
        } gguard{&graph, &gexec};
        int graph_fallbacks = 0;
        bool eager = !o->use_graph;
        auto run_batch = [&]() {
            if (grouped) {
                const rr_status rs = runner->run(Bt, X, ldx);
                if (rs != RR_OK) throw RrError{rs, "grouped PCG replay failed on the device"};
                return;
            }
            if (eager) {
                for (int k = 0; k < o->check_every; ++k) Bt.iteration(X, ldx);
                return;
            }
            RR_HIP(hipStreamSynchronize(st));   // everything queued on st precedes the replay
            if (!gexec) {
                cap = capture.get();
                Bt.st = cap;
                // relaxed: the capture holds kernel launches only, and allocation or copy calls
                // of other threads (a server's other requests) must not invalidate it
                RR_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
                for (int k = 0; k < o->check_every; ++k) Bt.iteration(X, ldx);
                const hipError_t ce = hipStreamEndCapture(cap, &graph);
                Bt.st = st;
                if (ce != hipSuccess) {
                    // An invalidated capture has run nothing: the batch runs eagerly, now
                    // and for the rest of the solve, with the same kernels and results,
                    // and every column's info.graph_fallbacks reports it.
                    (void)hipGetLastError();
                    if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
                    eager = true;
                    graph_fallbacks = 1;
                    for (int k = 0; k < o->check_every; ++k) Bt.iteration(X, ldx);
                    return;
                }
                RR_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
            }
            RR_HIP(hipGraphLaunch(gexec, cap));
            RR_HIP(hipStreamSynchronize(cap));
        };
        bool running = restart_pass();
        while (running) {
            run_batch();
            RR_HIP(hipGetLastError());
            RR_HIP(hipMemcpyAsync(hs.data(), Bt.state.ptr(), m * sizeof(BState), hipMemcpyDeviceToHost, st));
            RR_HIP(hipStreamSynchronize(st));
            int active = 0, need = 0;
            for (int64_t j = 0; j < m; ++j) {
                if (done[j]) continue;
                iters[j] = hs[j].iters;
                if (hs[j].run) { ++active; continue; }
                if (hs[j].code == STOP_BREAKDOWN) { done[j] = 1; status[j] = RR_EBREAKDOWN; continue; }
                if (!pending[j]) { pending[j] = 1; ++need; }
            }
            if (need > 0) {
                const bool started = restart_pass();
                if (!started && active == 0) break;
            } else if (active == 0) {
                break;
            }
        }
        const double t_solve = now_ms() - t0;
        std::vector<double> rel64(m, std::nan(""));
        if (ir || P.opts.prec == RR_PREC_FP64) {
            // every column's last true residual came from the float64 operator
            rel64 = relres;
        } else if (o->certify) {
            Bt.matmat(X, ldx, Bt.T.as<double>(), true);
            launch_bresid(n, m, B, ldb, Bt.T.as<double>(), Bt.T.as<double>(), st);
            const std::vector<double> rr = Bt.coldots(Bt.T.as<double>(), n, Bt.T.as<double>(), n);
            for (int64_t j = 0; j < m; ++j) rel64[j] = nb[j] > 0 ? std::sqrt(rr[j]) / nb[j] : 0.0;
        }
        rr_status first = RR_OK;
        for (int64_t j = 0; j < m; ++j) {
            if (!done[j]) status[j] = RR_ENOCONV;
            if (status[j] != RR_OK && first == RR_OK) first = (rr_status)status[j];
            if (infos) {
                rr_solve_info& inf = infos[j];
                const PerMu& pm = P.per[mu_index_per_col[j]];
                inf.iters = iters[j];
                inf.graph_fallbacks = graph_fallbacks;
                inf.restarts = std::max(cycles[j] - 1, 0);
                inf.relres_work = relres[j];
                inf.relres_fp64 = rel64[j];
                inf.tau = pm.tau; inf.normE = pm.normE; inf.lamhat = pm.lam;
                inf.orth_err = P.orth_err;
                inf.ms_build = P.ms_build;
                inf.ms_solve = t_solve;
                inf.status = status[j];
            }
        }
        if (first != RR_OK) set_error("at least one column did not converge (see infos)");
        return first;
    });
}
