// Block Krylov solves of rr_solve_batch (krylov BLOCK_MINRES / BLOCK_CG): the columns
// under one shift, in groups of at most BLOCK_MAX_S, each solved as one block with
// the C-RandRAND preconditioner (Section 7.2.2: block preconditioned MINRES with a
// reorthogonalised Krylov basis; convergence on max_i ||b_i - A_mu x_i|| / ||b_i||).
//
// Block MINRES, per step k on the block of s active columns:
//   U = A_mu Z_k;  W = U - V_{k-1} C_k^T;  M = sym(Z_k^T W);  W -= V_k M
//   W -= V (Z^T W) over every stored block, twice (full reorthogonalisation)
//   Zt = P W;  W^T Zt = C_{k+1}^T C_{k+1};  V_{k+1} = W C_{k+1}^{-1}, Z_{k+1} = Zt C_{k+1}^{-1}
//   block QR step of T_k (k_bmr_qr), then D_k, A_mu D_k, Y, R (k_bmr_rows).
// Block CG, per step: D = P R made A_mu-orthogonal to every stored block (twice),
//   A_mu D, D^T A_mu D = L^T L, D <- D L^{-1}, A_mu D <- A_mu D L^{-1},
//   a = D^T R, Y += D a, R -= A_mu D a.
// Restarts as in the single solve (Algorithm RandRAND_PCG step 10 with eta): every
// cycle starts from the true residual block (the float64 operator under
// refinement), keeps only the columns not yet at tol and ends when each kept column
// reaches max(eta ||r_i||, tol ||b_i||), or after block_kmax steps (the storage of
// the reorthogonalisation).  The host reads the column norms after every step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

using namespace rr;

namespace {

enum { CYC_OK = 0, CYC_BREAKDOWN = 1, CYC_LIMIT = 2 };

struct BlockSolver {
    const rr_precond& P;
    hipStream_t st;
    int64_t n;
    int s0;          // columns of the group
    int kmax;        // steps per cycle
    bool minres;
    Batch Bt;
    const Alloc* al;
    DBuf V, Z, U, W, Zt, D[3], AD[3], Yc, Rc, H;
    DBuf sm;         // small matrices
    DBuf flag, idx;
    // small-matrix slots (s0 x s0 each, G slots 2 s0 x 2 s0)
    double *M, *S, *C[2], *Ci, *phibar, *R1, *R2, *Rinv, *phi, *G[3], *a;

    BlockSolver(const rr_precond& p, hipStream_t s, int64_t ncols, int km, bool mr)
        : P(p), st(s), n(p.n), s0((int)ncols), kmax(km), minres(mr), Bt(p, s, ncols), al(Bt.al) {
        const size_t blk = (size_t)n * s0 * sizeof(double);
        const int nstore = minres ? kmax + 1 : kmax;
        V.reset(al, blk * nstore);
        Z.reset(al, blk * nstore);
        U.reset(al, blk); W.reset(al, blk); Zt.reset(al, blk); Yc.reset(al, blk); Rc.reset(al, blk);
        if (minres)
            for (int i = 0; i < 3; ++i) { D[i].reset(al, blk); AD[i].reset(al, blk); }
        H.reset(al, (size_t)(kmax + 1) * s0 * s0 * sizeof(double));
        const size_t ss = (size_t)s0 * s0;
        sm.reset(al, (11 + 3 * 4) * ss * sizeof(double));
        double* q = sm.as<double>();
        auto take = [&](size_t k) { double* r = q; q += k; return r; };
        M = take(ss); S = take(ss); C[0] = take(ss); C[1] = take(ss); Ci = take(ss);
        phibar = take(ss); R1 = take(ss); R2 = take(ss); Rinv = take(ss); phi = take(ss); a = take(ss);
        for (int i = 0; i < 3; ++i) G[i] = take(4 * ss);
        flag.reset(al, 16);
        idx.reset(al, (size_t)s0 * sizeof(int32_t));
    }

    void gemm(bool ta, bool tb, int64_t Mr, int64_t Nc, int64_t K, const double* A, int64_t lda,
              const double* B, int64_t ldb, double* Cm, int64_t ldc, double alpha, double beta) {
        Bt.gemm(ta, tb, Mr, Nc, K, A, lda, B, ldb, Cm, ldc, alpha, beta);
    }
    double* slot(const DBuf& b, int k, int s) const { return b.as<double>() + (size_t)k * n * s; }

    int32_t read_flag_and_norms(int s, std::vector<double>& rn) {
        int32_t f = 0;
        RR_HIP(hipMemcpyAsync(&f, flag.ptr(), sizeof(int32_t), hipMemcpyDeviceToHost, st));
        Bt.m = s;
        const std::vector<double> c2 = Bt.coldots(Rc.as<double>(), n, Rc.as<double>(), n);   // syncs
        rn.resize(s);
        for (int j = 0; j < s; ++j) rn[j] = std::sqrt(c2[j]);
        return f;
    }

    bool met(const std::vector<double>& rn, const std::vector<double>& tg) const {
        for (size_t j = 0; j < rn.size(); ++j)
            if (!(rn[j] <= tg[j])) return false;
        return true;
    }

    // One cycle on the s columns held in Rc (the residual block, updated in place);
    // the correction accumulates in Yc.  Returns CYC_* and the steps taken.
    int cycle_minres(int s, const std::vector<double>& tg, int maxsteps, int& steps) {
        Bt.m = s;
        double* w = W.as<double>();
        double* zt = Zt.as<double>();
        double* u = U.as<double>();
        RR_HIP(hipMemsetAsync(flag.ptr(), 0, sizeof(int32_t), st));
        RR_HIP(hipMemsetAsync(Yc.ptr(), 0, (size_t)n * s * sizeof(double), st));
        launch_copy_mat(DT_F64, Rc.ptr(), n, DT_F64, w, n, n, s, st);
        Bt.precond(w, zt);
        gemm(true, false, s, s, n, w, n, zt, n, S, s, 1.0, 0.0);
        launch_blk_chol(s, S, phibar, Ci, flag.as<int32_t>(), st);   // phibar_1 = C_1
        int32_t f = 0;
        RR_HIP(hipMemcpyAsync(&f, flag.ptr(), sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RR_HIP(hipStreamSynchronize(st));
        steps = 0;
        if (f) return CYC_BREAKDOWN;
        gemm(false, false, n, s, s, w, n, Ci, s, slot(V, 0, s), n, 1.0, 0.0);
        gemm(false, false, n, s, s, zt, n, Ci, s, slot(Z, 0, s), n, 1.0, 0.0);
        std::vector<double> rn;
        int cur = 0;   // C[cur] = C_k (from the previous step)
        for (int k = 0; k < maxsteps; ++k) {
            const double* Vk = slot(V, k, s);
            const double* Zk = slot(Z, k, s);
            Bt.matmat(Zk, n, u, false);
            launch_copy_mat(DT_F64, u, n, DT_F64, w, n, n, s, st);
            if (k > 0) gemm(false, true, n, s, s, slot(V, k - 1, s), n, C[cur], s, w, n, -1.0, 1.0);
            gemm(true, false, s, s, n, Zk, n, w, n, M, s, 1.0, 0.0);
            launch_symmetrize(M, s, s, st);
            gemm(false, false, n, s, s, Vk, n, M, s, w, n, -1.0, 1.0);
            const int64_t kk = (int64_t)(k + 1) * s;
            for (int pass = 0; pass < 2; ++pass) {
                gemm(true, false, kk, s, n, Z.as<double>(), n, w, n, H.as<double>(), kk, 1.0, 0.0);
                gemm(false, false, n, s, kk, V.as<double>(), n, H.as<double>(), kk, w, n, -1.0, 1.0);
            }
            Bt.precond(w, zt);
            gemm(true, false, s, s, n, w, n, zt, n, S, s, 1.0, 0.0);
            double* Cn = C[cur ^ 1];
            launch_blk_chol(s, S, Cn, Ci, flag.as<int32_t>(), st);
            if (k + 1 <= kmax) {
                gemm(false, false, n, s, s, w, n, Ci, s, slot(V, k + 1, s), n, 1.0, 0.0);
                gemm(false, false, n, s, s, zt, n, Ci, s, slot(Z, k + 1, s), n, 1.0, 0.0);
            }
            launch_bmr_qr(s, k, M, C[cur], Cn, flag.as<int32_t>(), G[(k + 1) % 3], G[(k + 2) % 3], G[k % 3],
                          phibar, R2, R1, Rinv, phi, st);
            const double* d1 = k >= 1 ? D[(k + 2) % 3].as<double>() : nullptr;
            const double* d2 = k >= 2 ? D[(k + 1) % 3].as<double>() : nullptr;
            const double* a1 = k >= 1 ? AD[(k + 2) % 3].as<double>() : nullptr;
            const double* a2 = k >= 2 ? AD[(k + 1) % 3].as<double>() : nullptr;
            launch_bmr_rows(n, s, Zk, u, d1, d2, a1, a2, R1, R2, Rinv, phi, D[k % 3].as<double>(),
                            AD[k % 3].as<double>(), Yc.as<double>(), Rc.as<double>(), st);
            RR_HIP(hipGetLastError());
            f = read_flag_and_norms(s, rn);
            steps = k + 1;
            if (met(rn, tg)) return CYC_OK;
            if (f) return CYC_BREAKDOWN;
            cur ^= 1;
        }
        return CYC_LIMIT;
    }

    int cycle_cg(int s, const std::vector<double>& tg, int maxsteps, int& steps) {
        Bt.m = s;
        double* dt = W.as<double>();
        double* adt = U.as<double>();
        RR_HIP(hipMemsetAsync(flag.ptr(), 0, sizeof(int32_t), st));
        RR_HIP(hipMemsetAsync(Yc.ptr(), 0, (size_t)n * s * sizeof(double), st));
        std::vector<double> rn;
        steps = 0;
        for (int k = 0; k < maxsteps; ++k) {
            Bt.precond(Rc.as<double>(), dt);
            const int64_t kk = (int64_t)k * s;
            if (k > 0)
                for (int pass = 0; pass < 2; ++pass) {
                    gemm(true, false, kk, s, n, Z.as<double>(), n, dt, n, H.as<double>(), kk, 1.0, 0.0);
                    gemm(false, false, n, s, kk, V.as<double>(), n, H.as<double>(), kk, dt, n, -1.0, 1.0);
                }
            Bt.matmat(dt, n, adt, false);
            gemm(true, false, s, s, n, dt, n, adt, n, S, s, 1.0, 0.0);
            launch_blk_chol(s, S, C[0], Ci, flag.as<int32_t>(), st);
            double* Dk = slot(V, k, s);     // V holds the directions D_j, Z their products A_mu D_j
            double* ADk = slot(Z, k, s);
            gemm(false, false, n, s, s, dt, n, Ci, s, Dk, n, 1.0, 0.0);
            gemm(false, false, n, s, s, adt, n, Ci, s, ADk, n, 1.0, 0.0);
            gemm(true, false, s, s, n, Dk, n, Rc.as<double>(), n, a, s, 1.0, 0.0);
            gemm(false, false, n, s, s, Dk, n, a, s, Yc.as<double>(), n, 1.0, 1.0);
            gemm(false, false, n, s, s, ADk, n, a, s, Rc.as<double>(), n, -1.0, 1.0);
            RR_HIP(hipGetLastError());
            const int32_t f = read_flag_and_norms(s, rn);
            if (f) return CYC_BREAKDOWN;     // C^{-1} = 0: nothing was updated
            steps = k + 1;
            if (met(rn, tg)) return CYC_OK;
        }
        return CYC_LIMIT;
    }
};

}  // namespace

rr_status rr_solve_block(const rr_precond* Pc, const int32_t* mu_index_per_col, const double* B, int64_t ldb,
                         int32_t nrhs, double* X, int64_t ldx, const rr_solve_opts* o, rr_solve_info* infos,
                         void* hip_stream) {
    if (infos)
        for (int j = 0; j < nrhs; ++j) { std::memset(&infos[j], 0, sizeof(rr_solve_info)); infos[j].status = RR_EINVAL; }
    return guarded([&]() -> rr_status {
        require_device();
        const rr_precond& P = *Pc;
        hipStream_t st = (hipStream_t)hip_stream;
        const int64_t n = P.n, m = nrhs;
        const double t0 = now_ms();
        const bool minres = o->krylov == RR_KRYLOV_BLOCK_MINRES;
        const bool ir = (o->fp64_ir == 1) || (o->fp64_ir == -1 && P.opts.prec != RR_PREC_FP64);
        {
            Alloc alloc = P.alloc;
            alloc.st = st;
            DBuf fl(&alloc, 16);
            RR_HIP(hipMemsetAsync(fl.ptr(), 0, 2 * sizeof(int32_t), st));
            for (int64_t j = 0; j < m; ++j) {
                launch_nonfinite(n, B + j * ldb, fl.as<int32_t>(), st);
                launch_nonfinite(n, X + j * ldx, fl.as<int32_t>(), st);
            }
            int32_t h = 0;
            RR_HIP(hipMemcpyAsync(&h, fl.ptr(), sizeof(int32_t), hipMemcpyDeviceToHost, st));
            RR_HIP(hipStreamSynchronize(st));
            RR_REQUIRE(h == 0, "B or X0 contains NaN or Inf");
        }
        // groups: columns of one shift in order, at most BLOCK_MAX_S per group
        std::vector<std::vector<int32_t>> groups;
        for (size_t g = 0; g < P.per.size(); ++g) {
            std::vector<int32_t> cols;
            for (int64_t j = 0; j < m; ++j)
                if (mu_index_per_col[j] == (int32_t)g) cols.push_back((int32_t)j);
            for (size_t c0 = 0; c0 < cols.size(); c0 += BLOCK_MAX_S)
                groups.emplace_back(cols.begin() + c0,
                                    cols.begin() + std::min(cols.size(), c0 + (size_t)BLOCK_MAX_S));
        }
        std::vector<int> status(m, RR_ENOCONV), iters(m, 0), restarts(m, 0);
        std::vector<double> relres(m, 1.0);
        for (const std::vector<int32_t>& gc : groups) {
            const int s0 = (int)gc.size();
            const int g = mu_index_per_col[gc[0]];
            const double mu = P.per[g].mu;
            BlockSolver bs(P, st, s0, o->block_kmax, minres);
            Batch& Bt = bs.Bt;
            Bt.mus_used = {g};
            Bt.setup_single_shift();
            const std::vector<double> hmu(s0, mu);
            const std::vector<int32_t> hidx(s0, g);
            RR_HIP(hipMemcpyAsync(Bt.mucol.ptr(), hmu.data(), s0 * sizeof(double), hipMemcpyHostToDevice, st));
            RR_HIP(hipMemcpyAsync(Bt.muidx.ptr(), hidx.data(), s0 * sizeof(int32_t), hipMemcpyHostToDevice, st));
            // group's B and X as contiguous n x s0 blocks (Bt.R holds B, Bt.Pm holds X)
            double* Bg = Bt.R.as<double>();
            double* Xg = Bt.Pm.as<double>();
            double* Tg = Bt.T.as<double>();
            RR_HIP(hipMemcpyAsync(bs.idx.ptr(), gc.data(), s0 * sizeof(int32_t), hipMemcpyHostToDevice, st));
            launch_blk_gather(n, s0, B, ldb, bs.idx.as<int32_t>(), Bg, st);
            launch_blk_gather(n, s0, X, ldx, bs.idx.as<int32_t>(), Xg, st);
            Bt.m = s0;
            const std::vector<double> bb = Bt.coldots(Bg, n, Bg, n);
            std::vector<double> nb(s0), rel(s0, 1.0);
            for (int j = 0; j < s0; ++j) nb[j] = std::sqrt(bb[j]);
            int its = 0, cycles = 0, gstat = RR_ENOCONV;
            while (true) {
                Bt.m = s0;
                Bt.matmat(Xg, n, Tg, ir);
                launch_bresid(n, s0, Bg, n, Tg, Tg, st);
                const std::vector<double> rr = Bt.coldots(Tg, n, Tg, n);
                std::vector<int32_t> act;
                std::vector<double> tg;
                for (int j = 0; j < s0; ++j) {
                    const double rn = std::sqrt(rr[j]);
                    rel[j] = nb[j] > 0.0 ? rn / nb[j] : 0.0;
                    RR_REQUIRE(std::isfinite(rn), "non-finite residual in a block solve");
                    if (nb[j] > 0.0 && rn > o->tol * nb[j]) {
                        act.push_back(j);
                        tg.push_back(std::max(o->restart_eta * rn, o->tol * nb[j]));
                    }
                }
                if (act.empty()) { gstat = RR_OK; break; }
                if (its >= o->maxit) { gstat = RR_ENOCONV; break; }
                ++cycles;
                const int s = (int)act.size();
                RR_HIP(hipMemcpyAsync(bs.idx.ptr(), act.data(), s * sizeof(int32_t), hipMemcpyHostToDevice, st));
                launch_blk_gather(n, s, Tg, n, bs.idx.as<int32_t>(), bs.Rc.as<double>(), st);
                int steps = 0;
                const int left = std::min(o->maxit - its, bs.kmax);
                const int c = minres ? bs.cycle_minres(s, tg, left, steps) : bs.cycle_cg(s, tg, left, steps);
                launch_blk_scatter(n, s, bs.Yc.as<double>(), bs.idx.as<int32_t>(), Xg, n, true, st);
                its += steps;
                if (c == CYC_BREAKDOWN && steps == 0) {
                    Bt.m = s0;
                    Bt.matmat(Xg, n, Tg, ir);
                    launch_bresid(n, s0, Bg, n, Tg, Tg, st);
                    const std::vector<double> r2 = Bt.coldots(Tg, n, Tg, n);
                    for (int j = 0; j < s0; ++j) rel[j] = nb[j] > 0.0 ? std::sqrt(r2[j]) / nb[j] : 0.0;
                    gstat = RR_EBREAKDOWN;
                    break;
                }
            }
            RR_HIP(hipMemcpyAsync(bs.idx.ptr(), gc.data(), s0 * sizeof(int32_t), hipMemcpyHostToDevice, st));
            launch_blk_scatter(n, s0, Xg, bs.idx.as<int32_t>(), X, ldx, false, st);
            RR_HIP(hipStreamSynchronize(st));
            for (int j = 0; j < s0; ++j) {
                const int col = gc[j];
                iters[col] = its;
                restarts[col] = std::max(cycles - 1, 0);
                relres[col] = rel[j];
                status[col] = (nb[j] == 0.0 || rel[j] <= o->tol) ? RR_OK : gstat;
            }
        }
        const double t_solve = now_ms() - t0;
        std::vector<double> rel64(m, std::nan(""));
        if (ir || P.opts.prec == RR_PREC_FP64) {
            rel64 = relres;
        } else if (o->certify) {
            Batch Bc(P, st, m);
            std::vector<double> hmu(m);
            for (int64_t j = 0; j < m; ++j) hmu[j] = P.per[mu_index_per_col[j]].mu;
            RR_HIP(hipMemcpyAsync(Bc.mucol.ptr(), hmu.data(), m * sizeof(double), hipMemcpyHostToDevice, st));
            Bc.matmat(X, ldx, Bc.T.as<double>(), true);
            launch_bresid(n, m, B, ldb, Bc.T.as<double>(), Bc.T.as<double>(), st);
            const std::vector<double> rr = Bc.coldots(Bc.T.as<double>(), n, Bc.T.as<double>(), n);
            const std::vector<double> bb = Bc.coldots(B, ldb, B, ldb);
            for (int64_t j = 0; j < m; ++j) rel64[j] = bb[j] > 0 ? std::sqrt(rr[j] / bb[j]) : 0.0;
        }
        rr_status first = RR_OK;
        for (int64_t j = 0; j < m; ++j) {
            if (status[j] != RR_OK && first == RR_OK) first = (rr_status)status[j];
            if (infos) {
                rr_solve_info& inf = infos[j];
                const PerMu& pm = P.per[mu_index_per_col[j]];
                inf.iters = iters[j];
                inf.restarts = restarts[j];
                inf.relres_work = relres[j];
                inf.relres_fp64 = rel64[j];
                inf.tau = pm.tau; inf.normE = pm.normE; inf.lamhat = pm.lam;
                inf.orth_err = P.orth_err;
                inf.ms_build = P.ms_build;
                inf.ms_solve = t_solve;
                inf.status = status[j];
            }
        }
        if (first != RR_OK) set_error("a block did not converge (see infos)");
        return first;
    });
}
