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

#include "ctx.hpp"

using namespace rr;

namespace {

constexpr int64_t KMULTI_MAX = 32;

struct Batch {
    const rr_precond& P;
    hipStream_t st;
    int64_t n, m, kb;
    Alloc alloc;          // the handle's allocator, ordered on the solve stream
    const Alloc* al;
    DBuf R, Pm, Z, W, T, parts, C, Dall, D, state, start, target2, mucol, muidx, gws;
    DBuf kws, kdot;       // symmetric multi-column kernel matvec (few columns)
    bool kmulti = false;
    DBuf cpart, dcols, rzp;   // projection through the basis, groups of up to 8 columns
    int pmax = 0, gch = 1;
    DBuf rrp;                 // block partials of ||r_j||^2 from the x, r update
    DBuf cnt;                 // per-column block counters of the fused updates (2 m int32)
    bool single = false;      // every column under one shift mu1
    double mu1 = 0.0;
    size_t gwsd = 0;
    std::vector<int> mus_used;
    int nch = 1;

    Batch(const rr_precond& p, hipStream_t s, int64_t mcols)
        : P(p), st(s), n(p.n), m(mcols), kb(p.kb), alloc(p.alloc), al(&alloc) {
        alloc.st = s;
        const size_t nm = (size_t)n * m * sizeof(double);
        R.reset(al, nm); Pm.reset(al, nm); Z.reset(al, nm); W.reset(al, nm); T.reset(al, nm);
        nch = coldot_chunks(n);
        parts.reset(al, (size_t)nch * m * sizeof(double));
        if (kb > 0) {
            C.reset(al, (size_t)kb * m * sizeof(double));
            D.reset(al, (size_t)kb * m * sizeof(double));
            Dall.reset(al, (size_t)p.per.size() * kb * m * sizeof(double));
        }
        state.reset(al, (size_t)m * sizeof(BState));
        start.reset(al, (size_t)m * sizeof(int32_t));
        target2.reset(al, (size_t)m * sizeof(double));
        mucol.reset(al, (size_t)m * sizeof(double));
        muidx.reset(al, (size_t)m * sizeof(int32_t));
        gwsd = std::max<size_t>((size_t)8 * std::max<int64_t>(kb, 1) * m, (size_t)1 << 20);
        gws.reset(al, gwsd * sizeof(double));
        // a few columns: the symmetric matvec kernel (each entry formed once per
        // group of up to 8 columns, float64 sums) beats a 128-column MFMA tile
        kmulti = is_kernel(p.op) && p.opts.prec != RR_PREC_FP64 && m <= KMULTI_MAX;
        if (kmulti) {
            kws.reset(al, (kernel_matvec_ws_doubles(n, p.op.d, (int)std::min<int64_t>(m, 8)) + 1) * sizeof(double));
            kdot.reset(al, (size_t)kernel_matvec_blocks(n) * m * sizeof(double));
        }
        rrp.reset(al, (size_t)bxr_blocks(n) * m * sizeof(double));
        cnt.reset(al, (size_t)2 * m * sizeof(int32_t));
        RR_HIP(hipMemsetAsync(state.ptr(), 0, (size_t)m * sizeof(BState), st));
        RR_HIP(hipMemsetAsync(cnt.ptr(), 0, (size_t)2 * m * sizeof(int32_t), st));
    }

    // Few columns under one shift: the projection is a streaming pass over Qb per
    // group of columns (Qb^T R, the core, R + Qb D) rather than GEMMs, which cuts
    // the launches per iteration.  Group width limited by the qd kernel's LDS
    // (D of the group plus its partial sums within 64 KiB).
    // A single shift also folds mu into the kernel product, whose block partials
    // of p_j^T w_j then serve alpha, and the projection's partials of r_j^T z_j
    // serve beta (no separate column dots).
    void setup_single_shift() {
        if (mus_used.size() != 1) return;
        single = true;
        mu1 = P.per[mus_used[0]].mu;
        if (kb == 0 || m > KMULTI_MAX) return;
        pmax = kb <= 768 ? 8 : kb <= 1792 ? 4 : 0;
        if (pmax == 0) return;
        gch = gemv_t_chunks(n, kb);
        cpart.reset(al, (size_t)pmax * gch * kb * sizeof(double));
        dcols.reset(al, (size_t)pmax * kb * sizeof(double));
        rzp.reset(al, (size_t)m * qd_blocks(n) * sizeof(double));
    }

    void gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
              const void* B, int64_t ldb, double* Cm, int64_t ldc, double alpha, double beta,
              int dta = DT_F64) {
        launch_gemm(dta, ta, DT_F64, tb, M, N, K, A, lda, B, ldb, Cm, ldc, alpha, beta, gws.as<double>(), gwsd, st);
    }

    // Wout = A_mu Pin for every column (fp64: float64 operator).  Returns the block
    // partials of Pin_j^T Wout_j when the product produced them (nch = 0 otherwise).
    ColParts matmat(const double* Pin, int64_t ldp, double* Wout, bool fp64) {
        if (kmulti && fp64 && ldp == n) {
            // a few columns under the float64 operator: the pair-once float64 matvec,
            // two columns per pass
            const KernelOp k = kernel_op_of(P);
            launch_kernel_matvec_multi(k, true, Pin, (int)m, 0.0, Wout, kdot.as<double>(), kws.as<double>(),
                                       nullptr, st);
            launch_add_shift_cols(n, m, mucol.as<double>(), Pin, ldp, Wout, n, st);
            return ColParts{nullptr, 0, 0, 0};
        }
        if (kmulti && !fp64 && ldp == n) {
            const KernelOp k = kernel_op_of(P);
            const int nblk = kernel_matvec_blocks(n);
            launch_kernel_matvec_multi(k, false, Pin, (int)m, single ? mu1 : 0.0, Wout, kdot.as<double>(),
                                       kws.as<double>(), nullptr, st);
            if (single) return ColParts{kdot.as<double>(), nblk, 1, nblk};
            launch_add_shift_cols(n, m, mucol.as<double>(), Pin, ldp, Wout, n, st);
            return ColParts{nullptr, 0, 0, 0};
        }
        if (is_kernel(P.op)) {
            const KernelOp k = kernel_op_of(P);
            launch_kernel_matmat_f64(k, fp64 || P.opts.prec == RR_PREC_FP64, mucol.as<double>(), Pin, ldp, m,
                                     Wout, n, st);
        } else {
            if (!fp64 && P.A32.ptr()) gemm(false, false, n, m, n, P.A32.ptr(), n, Pin, ldp, Wout, n, 1.0, 0.0, DT_F32);
            else gemm(false, false, n, m, n, P.op.A, P.op.lda, Pin, ldp, Wout, n, 1.0, 0.0);
            launch_add_shift_cols(n, m, mucol.as<double>(), Pin, ldp, Wout, n, st);
        }
        return ColParts{nullptr, 0, 0, 0};
    }

    // Zout = P_{mu(j)} Rin for every column.  Returns the block partials of
    // Rin_j^T Zout_j when the projection produced them (nch = 0 otherwise).
    ColParts precond(const double* Rin, double* Zout) {
        const double* Qb = P.Qb.as<double>();
        if (pmax > 0) {
            const double* Kc = P.per[mus_used[0]].Kc.as<double>();
            const int nb = qd_blocks(n);
            for (int64_t c0 = 0; c0 < m;) {
                const int64_t left = m - c0;
                const int nr = left >= pmax ? pmax : left >= 4 ? 4 : left >= 2 ? 2 : 1;
                launch_gemv_t_multi(nr, n, kb, Qb, n, Rin + c0 * n, n, cpart.as<double>(), gch, nullptr, st);
                launch_core_apply_cols(kb, Kc, kb, cpart.as<double>(), gch, nr, dcols.as<double>(), st);
                launch_qd_multi(nr, n, kb, Qb, n, dcols.as<double>(), Rin + c0 * n, n, 1.0, 1.0, Zout + c0 * n,
                                rzp.as<double>() + c0 * nb, nullptr, st);
                c0 += nr;
            }
            return ColParts{rzp.as<double>(), nb, 1, nb};
        }
        launch_copy_mat(DT_F64, Rin, n, DT_F64, Zout, n, n, m, st);
        if (kb == 0) return ColParts{nullptr, 0, 0, 0};
        gemm(true, false, kb, m, n, Qb, n, Rin, n, C.as<double>(), kb, 1.0, 0.0);
        for (int g : mus_used)
            gemm(false, false, kb, m, kb, P.per[g].Kc.ptr(), kb, C.ptr(), kb,
                 Dall.as<double>() + (size_t)g * kb * m, kb, 1.0, 0.0);
        launch_select_cols(kb, m, Dall.as<double>(), muidx.as<int32_t>(), D.as<double>(), st);
        gemm(false, false, n, m, kb, Qb, n, D.ptr(), kb, Zout, n, 1.0, 1.0);
        return ColParts{nullptr, 0, 0, 0};
    }

    // per-column sums of A_j^T B_j on the host (fixed order)
    std::vector<double> coldots(const double* A, int64_t lda, const double* B, int64_t ldb) {
        launch_coldot(n, m, A, lda, B, ldb, parts.as<double>(), st);
        std::vector<double> h((size_t)nch * m), out((size_t)m, 0.0);
        RR_HIP(hipMemcpyAsync(h.data(), parts.ptr(), h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        RR_HIP(hipStreamSynchronize(st));
        for (int64_t j = 0; j < m; ++j)
            for (int c = 0; c < nch; ++c) out[j] += h[(size_t)c * m + j];
        return out;
    }

    void iteration(double* X, int64_t ldx) {
        BState* s = state.as<BState>();
        double* r = R.as<double>();
        double* p = Pm.as<double>();
        double* w = W.as<double>();
        double* z = Z.as<double>();
        double* pp = parts.as<double>();
        const ColParts own{pp, nch, m, 1};
        int32_t* c = cnt.as<int32_t>();
        ColParts pw = matmat(p, n, w, false);
        if (!pw.p) { launch_coldot(n, m, p, n, w, n, pp, st); pw = own; }
        launch_bxr_fused(n, m, X, ldx, r, p, w, s, pw, rrp.as<double>(), c, st);
        ColParts rz = precond(r, z);
        if (!rz.p) { launch_coldot(n, m, r, n, z, n, pp, st); rz = own; }
        launch_bp_fused(n, m, z, p, s, rz, c + m, st);
    }
};

}  // namespace

rr_status rr_solve_batch_fused(const rr_precond* Pc, const int32_t* mu_index_per_col,
                               const double* B, int64_t ldb, int32_t nrhs, double* X, int64_t ldx,
                               const rr_solve_opts* o, rr_solve_info* infos, void* hip_stream) {
    if (infos)
        for (int j = 0; j < nrhs; ++j) { std::memset(&infos[j], 0, sizeof(rr_solve_info)); infos[j].status = RR_EINVAL; }
    return guarded([&]() -> rr_status {
        require_device();
        const rr_precond& P = *Pc;
        hipStream_t st = (hipStream_t)hip_stream;
        const int64_t n = P.n, m = nrhs;
        const double t0 = now_ms();
        Batch Bt(P, st, m);
        // per-column shifts and the set of shifts in use
        std::vector<double> hmu(m);
        std::vector<int> used(P.per.size(), 0);
        for (int64_t j = 0; j < m; ++j) { hmu[j] = P.per[mu_index_per_col[j]].mu; used[mu_index_per_col[j]] = 1; }
        for (size_t g = 0; g < used.size(); ++g) if (used[g]) Bt.mus_used.push_back((int)g);
        Bt.setup_single_shift();
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
                Bt.matmat(Xd, ldx, Bt.T.as<double>(), ir);
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
