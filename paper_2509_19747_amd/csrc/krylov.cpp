// rr_solve for the methods beside C-RandRAND PCG (which solve.cpp runs with its
// fused kernels): a general Krylov engine whose iterations run entirely on the
// device in batches (device stop flag, optionally replayed as a hipGraph).
//
//  * C-RandRAND MINRES: preconditioned MINRES on A_mu x = b with
//    P = I + Q (tau T G T - T) Q^T (the MINRES branch of Algorithm RandRAND_PCG).
//  * R-RandRAND (Algorithm RandRAND_CG): CG or MINRES on
//    B = (I-Pi) A_mu (I-Pi) + tau Pi (eq. APdef2), Pi = Q T Q^T (eq. accurate_proj),
//    tau = ||E|| (eq. cnd_bound, rho = 1); per restart cycle the solution is
//    recovered as x += Omega R^{-1} T Q^T (tau y - A_mu (I-Pi) y) + (I-Pi) y
//    (eq. APdef3 with eq. projector).
//  * split R-RandRAND (Algorithm RandRAND_CG_split): CG or MINRES on
//    E y = (I-Pi)(I-Pi) b_c, E u = (I-Pi) A_mu u (eq. APdef2_reduced), then
//    x += Omega R^{-1} T Q^T (b_c - A_mu y) + y.
// Every cycle starts from the true residual b_c = b - A_mu x (the float64 operator
// under refinement) and stops when the recurrence residual, which is the residual
// of the recovered x in exact arithmetic, drops below max(eta ||b_c||, tol ||b||).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.hpp"

using namespace rr;

namespace {

struct Gen {
    const rr_precond& P;
    const PerMu& pm;
    hipStream_t st;
    Alloc al;
    int64_t n = 0, kb = 0;
    int method = RR_METHOD_C, krylov = RR_KRYLOV_CG;
    double mu = 0.0, tau = 0.0;
    int nch = 1;
    DBuf kws, op_part, vpart, rzp, cgs, mrs, scal;
    DBuf c1, c2, d, tv, tw;
    DBuf negT, tauT, MRt, gws;
    size_t gwsd = 0;
    DBuf y, r, p, w;                                  // CG
    DBuf v, av, t, r1, r2, z, mw, mw2, maw, maw2, res;  // MINRES
    DBuf rc, rhs, hist;
    int32_t hist_cap = 0;

    Gen(const rr_precond& p_, const PerMu& pm_, hipStream_t s, const rr_solve_opts& o)
        : P(p_), pm(pm_), st(s), al(p_.alloc) {
        if (!al.custom) al.st = s;
        n = P.n;
        kb = P.kb;
        method = o.method;
        krylov = o.krylov;
        mu = pm.mu;
        tau = pm.normE;
        const Alloc* a = &al;
        const size_t nb = (size_t)n * sizeof(double);
        kws.reset(a, (operator_ws_doubles(P) + 1) * sizeof(double));
        op_part.reset(a, ((size_t)operator_part_count(P) + 1) * sizeof(double));
        vpart.reset(a, ((size_t)vec_blocks(n) + 1) * sizeof(double));
        rzp.reset(a, ((size_t)std::max(qd_blocks(n), vec_blocks(n)) + 1) * sizeof(double));
        cgs.reset(a, sizeof(CgState));
        mrs.reset(a, sizeof(MrState));
        scal.reset(a, 8 * sizeof(double));
        tv.reset(a, nb);
        tw.reset(a, nb);
        rc.reset(a, nb);
        rhs.reset(a, nb);
        y.reset(a, nb);
        if (kb > 0) {
            nch = gemv_t_chunks(n, kb);
            c1.reset(a, (size_t)nch * kb * sizeof(double));
            c2.reset(a, (size_t)nch * kb * sizeof(double));
            d.reset(a, (size_t)kb * sizeof(double));
        }
        if (krylov == RR_KRYLOV_CG) {
            r.reset(a, nb); p.reset(a, nb); w.reset(a, nb);
        } else {
            v.reset(a, nb); av.reset(a, nb); t.reset(a, nb); r1.reset(a, nb); r2.reset(a, nb); z.reset(a, nb);
            mw.reset(a, nb); mw2.reset(a, nb); maw.reset(a, nb); maw2.reset(a, nb); res.reset(a, nb);
        }
        hist_cap = o.maxit + 2;
        hist.reset(a, (size_t)hist_cap * sizeof(double));
        if (method != RR_METHOD_C) {
            // -T, tau T and (R^{-1} T)^T (the recovery's A_mu^{-1} Pi = Omega R^{-1} T Q^T)
            const int64_t l = P.l;
            // the GEMMs here split K only as far as this workspace allows
            gwsd = (size_t)4 * l * l + (size_t)4 * n + ((size_t)1 << 16);
            gws.reset(a, gwsd * sizeof(double));
            negT.reset(a, (size_t)l * l * sizeof(double));
            tauT.reset(a, (size_t)l * l * sizeof(double));
            MRt.reset(a, (size_t)l * l * sizeof(double));
            DBuf Rinv(a, (size_t)l * l * sizeof(double));
            launch_axpby_mat(-1.0, pm.T.as<double>(), l, 0.0, pm.T.as<double>(), l, negT.as<double>(), l, l, l, st);
            launch_axpby_mat(tau, pm.T.as<double>(), l, 0.0, pm.T.as<double>(), l, tauT.as<double>(), l, l, l, st);
            launch_tri_inv_upper(pm.R.as<double>(), l, l, Rinv.as<double>(), l, st);
            launch_gemm(DT_F64, false, DT_F64, true, l, l, l, pm.T.ptr(), l, Rinv.ptr(), l, MRt.as<double>(), l,
                        1.0, 0.0, gws.as<double>(), gwsd, st);
            RR_HIP(hipStreamSynchronize(st));   // Rinv is released on return
        }
    }

    void sync() { RR_HIP(hipStreamSynchronize(st)); }
    const double* Q() const { return P.Qb.as<double>(); }

    // out = A_mu u (fp64: the float64 operator)
    void opA(const double* u, double* out, const int32_t* stop, bool fp64 = false) {
        apply_operator(P, u, mu, out, op_part.as<double>(), kws.as<double>(), fp64, stop, st);
    }
    // out = (I - Pi) u with Pi = Q T Q^T
    void comp(const double* u, double* out, const int32_t* stop) {
        launch_gemv_t(n, kb, Q(), n, u, c1.as<double>(), nch, stop, st);
        launch_core_apply(kb, negT.as<double>(), kb, c1.as<double>(), nch, d.as<double>(), stop, st);
        launch_qd(n, kb, Q(), n, d.as<double>(), u, 1.0, out, rzp.as<double>(), stop, st);
    }
    // out = B u = (I-Pi) A_mu (I-Pi) u + tau Pi u
    void opB(const double* u, double* out, const int32_t* stop) {
        comp(u, tv.as<double>(), stop);   // leaves Q^T u in c1
        opA(tv.as<double>(), tw.as<double>(), stop);
        launch_gemv_t(n, kb, Q(), n, tw.as<double>(), c2.as<double>(), nch, stop, st);
        launch_core_apply2(kb, tauT.as<double>(), negT.as<double>(), kb, c1.as<double>(), c2.as<double>(), nch,
                           d.as<double>(), stop, st);
        launch_qd(n, kb, Q(), n, d.as<double>(), tw.as<double>(), 1.0, out, rzp.as<double>(), stop, st);
    }
    // out = E u = (I-Pi) A_mu u
    void opE(const double* u, double* out, const int32_t* stop) {
        opA(u, tw.as<double>(), stop);
        comp(tw.as<double>(), out, stop);
    }
    void op(const double* u, double* out, const int32_t* stop) {
        if (method == RR_METHOD_R) opB(u, out, stop);
        else if (method == RR_METHOD_SPLIT_R) opE(u, out, stop);
        else opA(u, out, stop);
    }
    // z = P r (C-RandRAND) or r; partials of r^T z into part; returns their count
    int prec(const double* rr_, double* zz, double* part, const int32_t* stop) {
        if (method == RR_METHOD_C && P.l > 0)
            return apply_projected(P, pm.Kc.as<double>(), rr_, 1.0, zz, c1.as<double>(), d.as<double>(), part,
                                   stop, st);
        launch_copy_dot(n, rr_, zz, part, stop, st);
        return vec_blocks(n);
    }

    // ------------------------------------------------------------ CG
    void cg_init(const double* b_rhs, double target, int32_t maxit, int32_t iters) {
        RR_HIP(hipMemsetAsync(y.ptr(), 0, (size_t)n * sizeof(double), st));
        launch_copy_vec(n, b_rhs, r.as<double>(), st);
        launch_copy_vec(n, b_rhs, p.as<double>(), st);
        launch_dot_part(n, b_rhs, b_rhs, vpart.as<double>(), st);
        launch_state_init(cgs.as<CgState>(), vpart.as<double>(), vec_blocks(n), target * target, maxit, iters,
                          hist.as<double>(), hist_cap, st);
    }
    void cg_iter(hipStream_t s) {
        hipStream_t keep = st;
        st = s;
        CgState* cs = cgs.as<CgState>();
        const int32_t* stop = &cs->stop;
        op(p.as<double>(), w.as<double>(), stop);
        launch_dot_part_stop(n, p.as<double>(), w.as<double>(), vpart.as<double>(), stop, st);
        launch_scal_alpha(vpart.as<double>(), vec_blocks(n), cs, st);
        launch_xr_update(n, y.as<double>(), r.as<double>(), p.as<double>(), w.as<double>(), cs, vpart.as<double>(),
                         st);
        launch_scal_rr(vpart.as<double>(), vec_blocks(n), cs, st);
        launch_scal_beta(vpart.as<double>(), vec_blocks(n), cs, st);
        launch_p_update(n, r.as<double>(), p.as<double>(), cs, st);
        st = keep;
    }

    // -------------------------------------------------------- MINRES
    void mr_init(const double* b_rhs, double target, int32_t maxit, int32_t iters) {
        const size_t bytes = (size_t)n * sizeof(double);
        RR_HIP(hipMemsetAsync(y.ptr(), 0, bytes, st));
        RR_HIP(hipMemsetAsync(mw.ptr(), 0, bytes, st));
        RR_HIP(hipMemsetAsync(mw2.ptr(), 0, bytes, st));
        RR_HIP(hipMemsetAsync(maw.ptr(), 0, bytes, st));
        RR_HIP(hipMemsetAsync(maw2.ptr(), 0, bytes, st));
        launch_copy_vec(n, b_rhs, res.as<double>(), st);
        launch_copy_vec(n, b_rhs, r1.as<double>(), st);
        launch_copy_vec(n, b_rhs, r2.as<double>(), st);
        const int cnt = prec(b_rhs, z.as<double>(), rzp.as<double>(), nullptr);
        launch_mr_init(rzp.as<double>(), cnt, mrs.as<MrState>(), target * target, maxit, iters, hist.as<double>(),
                       hist_cap, st);
    }
    void mr_iter(hipStream_t s) {
        hipStream_t keep = st;
        st = s;
        MrState* ms = mrs.as<MrState>();
        const int32_t* stop = &ms->stop;
        launch_mr_v(n, z.as<double>(), v.as<double>(), ms, st);
        op(v.as<double>(), av.as<double>(), stop);
        launch_mr_t(n, av.as<double>(), r1.as<double>(), v.as<double>(), t.as<double>(), ms, vpart.as<double>(), st);
        launch_mr_alfa(vpart.as<double>(), vec_blocks(n), ms, st);
        launch_mr_shift(n, t.as<double>(), r1.as<double>(), r2.as<double>(), ms, st);
        const int cnt = prec(r2.as<double>(), z.as<double>(), rzp.as<double>(), stop);
        launch_mr_rot(rzp.as<double>(), cnt, ms, st);
        launch_mr_update(n, v.as<double>(), av.as<double>(), mw.as<double>(), mw2.as<double>(), maw.as<double>(),
                         maw2.as<double>(), y.as<double>(), res.as<double>(), ms, vpart.as<double>(), st);
        launch_mr_rr(vpart.as<double>(), vec_blocks(n), ms, st);
        st = keep;
    }

    // x += the recovered correction of this cycle (y: the cycle's Krylov solution)
    void recover(double* x) {
        const double* yy = y.as<double>();
        if (method == RR_METHOD_C) {
            launch_axpby_mat(1.0, x, n, 1.0, yy, n, x, n, n, 1, st);
            return;
        }
        const int64_t l = P.l;
        double* g = rhs.as<double>();
        if (method == RR_METHOD_R) {
            // u = (I-Pi) y; g = tau y - A_mu u; x += Omega R^{-1} T Q^T g + u
            comp(yy, tv.as<double>(), nullptr);
            opA(tv.as<double>(), tw.as<double>(), nullptr);
            launch_axpby_mat(tau, yy, n, -1.0, tw.as<double>(), n, g, n, n, 1, st);
        } else {
            // g = b_c - A_mu y; x += Omega R^{-1} T Q^T g + y
            opA(yy, tw.as<double>(), nullptr);
            launch_axpby_mat(1.0, rc.as<double>(), n, -1.0, tw.as<double>(), n, g, n, n, 1, st);
            launch_copy_vec(n, yy, tv.as<double>(), st);
        }
        launch_gemv_t(n, kb, Q(), n, g, c1.as<double>(), nch, nullptr, st);
        launch_core_apply(kb, MRt.as<double>(), l, c1.as<double>(), nch, d.as<double>(), nullptr, st);
        launch_gemm(P.omega_dt, false, DT_F64, false, n, 1, l, P.Omega.ptr(), n, d.ptr(), l, x, n, 1.0, 1.0,
                    gws.as<double>(), gwsd, st);
        launch_axpby_mat(1.0, x, n, 1.0, tv.as<double>(), n, x, n, n, 1, st);
    }
};

}  // namespace

// The general engine; options validated by rr_solve.
rr_status rr_solve_general(const rr_precond* Pc, int32_t mu_index, const double* b, double* x,
                           const rr_solve_opts& o, rr_solve_info* info, hipStream_t st) {
    const rr_precond& P = *Pc;
    const PerMu& pm = P.per[mu_index];
    if (o.method != RR_METHOD_C) {
        RR_REQUIRE(P.l > 0, "R-RandRAND methods need a sketch (l > 0)");
        RR_REQUIRE(!P.joint, "R-RandRAND methods need a single-shift handle");
        RR_REQUIRE(!P.basisless, "R-RandRAND methods need an explicit basis");
        RR_REQUIRE(P.l <= 4096, "R-RandRAND methods support l <= 4096");
        if (o.method == RR_METHOD_R)
            RR_REQUIRE(std::isfinite(pm.normE) && pm.normE > 0.0,
                       "R-RandRAND needs the ||E|| estimate: build with tau rule OPT or RHO");
    }
    Gen G(P, pm, st, o);
    const int64_t n = P.n;
    const bool ir = (o.fp64_ir == 1) || (o.fp64_ir == -1 && P.opts.prec != RR_PREC_FP64);

    RR_HIP(hipMemsetAsync(G.scal.ptr(), 0, 8 * sizeof(double), st));
    int32_t* flag = (int32_t*)G.scal.ptr();
    launch_nonfinite(n, b, flag, st);
    launch_nonfinite(n, x, flag, st, flag + 1);
    int32_t flags[2] = {0, 0};
    RR_HIP(hipMemcpyAsync(flags, flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    G.sync();
    RR_REQUIRE(flags[0] == 0, "b or x0 contains NaN or Inf");
    const bool x0_zero = flags[1] == 0;

    const double t0 = now_ms();
    launch_dot_part(n, b, b, G.vpart.as<double>(), st);
    launch_scal_set(G.vpart.as<double>(), vec_blocks(n), G.scal.as<double>() + 1, st);
    double bb = 0.0;
    RR_HIP(hipMemcpyAsync(&bb, G.scal.as<double>() + 1, sizeof(double), hipMemcpyDeviceToHost, st));
    G.sync();
    const double nb = std::sqrt(bb);
    rr_solve_info inf{};
    inf.tau = o.method == RR_METHOD_R ? pm.normE : pm.tau;
    inf.normE = pm.normE;
    inf.lamhat = pm.lam;
    inf.orth_err = P.orth_err;
    inf.ms_build = P.ms_build;
    if (nb == 0.0) {
        RR_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
        G.sync();
        inf.status = RR_OK;
        inf.relres_fp64 = 0.0;
        inf.ms_solve = now_ms() - t0;
        if (info) *info = inf;
        return RR_OK;
    }

    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    PooledStream cap;
    struct GraphGuard {
        hipGraphExec_t* e; hipGraph_t* g;
        ~GraphGuard() { if (*e) (void)hipGraphExecDestroy(*e); if (*g) (void)hipGraphDestroy(*g); }
    } gg{&gexec, &graph};
    bool graph_failed = false;
    const bool is_cg = o.krylov == RR_KRYLOV_CG;
    auto iterate = [&](hipStream_t s) {
        if (is_cg) G.cg_iter(s);
        else G.mr_iter(s);
    };

    int its = 0, cycles = 0;
    rr_status result = RR_ENOCONV;
    double relres = 1.0;
    std::vector<double> hbuf;
    double* rc = G.rc.as<double>();
    while (true) {
        double rn2 = 0.0;
        if (x0_zero && cycles == 0) {
            launch_copy_vec(n, b, rc, st);
            rn2 = bb;
        } else {
            G.opA(x, G.tw.as<double>(), nullptr, ir);
            launch_residual(n, b, G.tw.as<double>(), rc, G.vpart.as<double>(), st);
            launch_scal_set(G.vpart.as<double>(), vec_blocks(n), G.scal.as<double>() + 1, st);
            RR_HIP(hipMemcpyAsync(&rn2, G.scal.as<double>() + 1, sizeof(double), hipMemcpyDeviceToHost, st));
            G.sync();
        }
        const double rn = std::sqrt(rn2);
        relres = rn / nb;
        if (its < o.history_cap) o.relres_history[its] = relres;
        if (!std::isfinite(rn)) { result = RR_EBREAKDOWN; break; }
        if (rn <= o.tol * nb) { result = RR_OK; break; }
        if (its >= o.maxit) { result = RR_ENOCONV; break; }
        ++cycles;
        const double target = std::max(o.restart_eta * rn, o.tol * nb);
        const double* rhs = rc;
        if (o.method == RR_METHOD_SPLIT_R) {
            // b_p = (I-Pi)(I-Pi) b_c
            G.comp(rc, G.tv.as<double>(), nullptr);
            G.comp(G.tv.as<double>(), G.rhs.as<double>(), nullptr);
            rhs = G.rhs.as<double>();
        }
        if (is_cg) G.cg_init(rhs, target, o.maxit, its);
        else G.mr_init(rhs, target, o.maxit, its);
        RR_HIP(hipGetLastError());
        int32_t stop = 0, hits = its;
        while (true) {
            if (o.use_graph && !graph_failed) {
                hipStream_t cst = cap.get();
                G.sync();
                if (!gexec) {
                    RR_HIP(hipStreamBeginCapture(cst, hipStreamCaptureModeRelaxed));
                    for (int k = 0; k < o.check_every; ++k) iterate(cst);
                    if (hipStreamEndCapture(cst, &graph) != hipSuccess) {
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
                for (int k = 0; k < o.check_every; ++k) iterate(st);
            }
            RR_HIP(hipGetLastError());
            if (is_cg) {
                CgState hs{};
                RR_HIP(hipMemcpyAsync(&hs, G.cgs.ptr(), sizeof(CgState), hipMemcpyDeviceToHost, st));
                G.sync();
                stop = hs.stop;
                hits = hs.iters;
            } else {
                MrState hs{};
                RR_HIP(hipMemcpyAsync(&hs, G.mrs.ptr(), sizeof(MrState), hipMemcpyDeviceToHost, st));
                G.sync();
                stop = hs.stop;
                hits = hs.iters;
            }
            if (stop != STOP_NONE) break;
        }
        if (o.history_cap > 0 && hits > its) {
            const int a = its + 1, e = std::min(hits, o.history_cap - 1);
            if (e >= a) {
                hbuf.resize((size_t)(e - a + 1));
                RR_HIP(hipMemcpyAsync(hbuf.data(), G.hist.as<double>() + a, hbuf.size() * sizeof(double),
                                      hipMemcpyDeviceToHost, st));
                G.sync();
                for (int q = a; q <= e; ++q) o.relres_history[q] = std::sqrt(hbuf[q - a]) / nb;
            }
        }
        its = hits;
        if (stop == STOP_BREAKDOWN) { result = RR_EBREAKDOWN; break; }
        G.recover(x);
        RR_HIP(hipGetLastError());
    }
    inf.iters = its;
    inf.graph_fallbacks = graph_failed ? 1 : 0;
    inf.restarts = std::max(cycles - 1, 0);
    inf.relres_work = relres;
    inf.ms_solve = now_ms() - t0;
    inf.relres_fp64 = std::nan("");
    if (ir || P.opts.prec == RR_PREC_FP64) {
        inf.relres_fp64 = relres;
    } else if (o.certify) {
        G.opA(x, G.tw.as<double>(), nullptr, true);
        launch_residual(n, b, G.tw.as<double>(), rc, G.vpart.as<double>(), st);
        launch_scal_set(G.vpart.as<double>(), vec_blocks(n), G.scal.as<double>() + 1, st);
        double r2 = 0.0;
        RR_HIP(hipMemcpyAsync(&r2, G.scal.as<double>() + 1, sizeof(double), hipMemcpyDeviceToHost, st));
        G.sync();
        inf.relres_fp64 = std::sqrt(r2) / nb;
    }
    inf.status = result;
    if (info) *info = inf;
    if (result != RR_OK)
        set_error(result == RR_ENOCONV ? "maximum iterations reached"
                                       : "Krylov breakdown (a non-positive curvature or norm)");
    return result;
}
