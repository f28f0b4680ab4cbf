// rr_build_precond: C-RandRAND preconditioner construction on the device,
// following Algorithm RandRAND_PCG steps 1-4 (Section 6.2) with the explicit
// basis of Section 4.1:
//   Omega (Section 2) -> Y_mu = A Omega + mu Omega -> Y_mu = Q R by the
//   sketched Cholesky QR of Algorithm prec_chol_qr (or Algorithm chol_qr) ->
//   G = (R_Omega R^{-1})^T (R_Omega R^{-1}) with R_Omega^T R_Omega = Omega^T A_mu Omega
//   (remark after Algorithm RandRAND_PCG) -> T = 2I - Q^T Q (eq. accurate_proj)
//   -> tau (eq. c_randrand_tau / optimal_rho / nys_tau, power iterations) ->
//   apply core K = tau T G T - T, so that P = I + Q K Q^T.
// Several shifts share the joint basis Q_joint = orth([Omega, A Omega]) and a
// per-shift 2l x l reduced Householder QR (Section 5.1).
// Only status words and a handful of scalars travel to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "ctx.hpp"

using namespace rr;

namespace {

struct Builder {
    rr_precond& P;
    hipStream_t st;
    const Alloc* al;
    DBuf gws;
    size_t gwsd = 0;
    DBuf status;   // int32
    DBuf scal;     // doubles
    DBuf kws;      // kernel-matvec workspace
    DBuf vparts;   // partial sums
    const void* Ob = nullptr;   // bf16 copy of Omega (float32-mode kernel sketch)
    int64_t ldo = 0;

    Builder(rr_precond& p, hipStream_t s) : P(p), st(s), al(&p.alloc) {
        const int64_t kmax = std::max<int64_t>(2 * p.l, 1);
        gwsd = std::max<size_t>((size_t)4 * kmax * kmax, (size_t)1 << 22);
        gws.reset(al, gwsd * sizeof(double));
        status.reset(al, 64);
        scal.reset(al, 64 * sizeof(double));
        kws.reset(al, (operator_ws_doubles(p) + 1) * sizeof(double));
        const int parts = std::max({operator_part_count(p), qd_blocks(p.n), vec_blocks(p.n), 1});
        vparts.reset(al, (size_t)parts * sizeof(double));
    }

    void gemm(int dta, bool ta, int dtb, bool tb, int64_t M, int64_t N, int64_t K, const void* A,
              int64_t lda, const void* B, int64_t ldb, double* C, int64_t ldc, double alpha = 1.0,
              double beta = 0.0) {
        launch_gemm(dta, ta, dtb, tb, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, gws.as<double>(),
                    gwsd, st);
    }
    // C = op(A) B (float64) with B upper triangular and zero below the diagonal (an
    // inverse from launch_tri_inv_upper): the MFMA kernel skips the zero blocks
    void gemm_upper_b(bool ta, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* C, int64_t ldc) {
        if (!launch_gemm_upper_b(ta, M, N, K, A, lda, B, ldb, C, ldc, gws.as<double>(), gwsd, st))
            gemm(DT_F64, ta, DT_F64, false, M, N, K, A, lda, B, ldb, C, ldc);
    }
    // C = A^T A (A: K x M float64): symmetric MFMA product, else the general GEMM
    void gram(int64_t M, int64_t K, const double* A, int64_t lda, double* C, int64_t ldc) {
        if (!launch_gemm_ata(M, K, A, lda, C, ldc, gws.as<double>(), gwsd, st)) {
            gemm(DT_F64, true, DT_F64, false, M, M, K, A, lda, A, lda, C, ldc);
            launch_symmetrize(C, M, ldc, st);
        }
    }
    DBuf mat(int64_t rows, int64_t cols, size_t esz = sizeof(double)) {
        return DBuf(al, (size_t)rows * cols * esz);
    }
    void sync() { RR_HIP(hipStreamSynchronize(st)); }
    void check_launch() { RR_HIP(hipGetLastError()); }

    // In-place upper Cholesky of the l x l spd matrix A with the shift ladder of
    // Appendix C: on failure retry with A + alpha I, alpha in {1e-14,...,1e-1} * max_i A_ii.
    // chol_start enqueues the first attempt on stream s (copy keeps A for retries);
    // chol_finish reads its status word (a host wait on s only) and runs the ladder.
    void chol_start(double* A, int64_t l, double* copy, hipStream_t s, int32_t* stat, double* ws,
                    size_t wsd) {
        RR_HIP(hipMemcpyAsync(copy, A, (size_t)l * l * sizeof(double), hipMemcpyDeviceToDevice, s));
        RR_HIP(hipMemsetAsync(stat, 0, sizeof(int32_t), s));
        launch_cholesky_upper(A, l, l, stat, ws, wsd, s);
        check_launch();
    }
    // returns the shift alpha that the factored matrix carries (0: none)
    double chol_finish(double* A, int64_t l, const double* copy, hipStream_t s, int32_t* stat, double* ws,
                       size_t wsd) {
        int32_t h = 0;
        RR_HIP(hipMemcpyAsync(&h, stat, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        RR_HIP(hipStreamSynchronize(s));
        if (h == 0) return 0.0;
        std::vector<double> hc((size_t)l * l);
        RR_HIP(hipMemcpyAsync(hc.data(), copy, hc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        RR_HIP(hipStreamSynchronize(s));
        double wn = 0.0;
        for (int64_t i = 0; i < l; ++i) wn = std::max(wn, std::fabs(hc[(size_t)i + (size_t)i * l]));
        if (!(wn > 0.0) || !std::isfinite(wn)) throw RrError{RR_ENOTSPD, "Cholesky: matrix is zero or not finite"};
        for (int e = -14; e <= -1; ++e) {
            const double alpha = std::pow(10.0, e) * wn;
            RR_HIP(hipMemcpyAsync(A, copy, (size_t)l * l * sizeof(double), hipMemcpyDeviceToDevice, s));
            launch_add_diag(A, l, l, alpha, s);
            RR_HIP(hipMemsetAsync(stat, 0, sizeof(int32_t), s));
            launch_cholesky_upper(A, l, l, stat, ws, wsd, s);
            check_launch();
            RR_HIP(hipMemcpyAsync(&h, stat, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            RR_HIP(hipStreamSynchronize(s));
            if (h == 0) return alpha;
        }
        throw RrError{RR_ENOTSPD, "Cholesky failed after the whole shift ladder"};
    }
    double chol_ladder(double* A, int64_t l) {
        DBuf copy = mat(l, l);
        chol_start(A, l, copy.as<double>(), st, status.as<int32_t>(), gws.as<double>(), gwsd);
        return chol_finish(A, l, copy.as<double>(), st, status.as<int32_t>(), gws.as<double>(), gwsd);
    }

    // A second stream for work that does not depend on the main chain (its own
    // status word and GEMM workspace); side_begin orders it after everything queued
    // on the main stream so far, side_join makes the main stream wait for it.
    PooledStream side;
    hipStream_t st2 = nullptr;
    DBuf gws2, status2;
    void side_begin() {
        if (!st2) {
            st2 = side.get();
            gws2.reset(al, gwsd * sizeof(double));
            status2.reset(al, 64);
        }
        RR_HIP(hipEventRecord(side.ev_a(), st));
        RR_HIP(hipStreamWaitEvent(st2, side.ev_a(), 0));
    }
    void side_join() {
        RR_HIP(hipEventRecord(side.ev_b(), st2));
        RR_HIP(hipStreamWaitEvent(st, side.ev_b(), 0));
    }

    // Omega (n x l) into P.Omega.  In float32 mode for kernels and in mixed mode for
    // dense operators Omega is drawn in bf16 (SRHT entries are exact, Gaussian
    // entries are rounded once) so the bf16 MFMA sketch sees the test matrix
    // exactly; P.Omega then holds the same values in float32.
    DBuf ob_buf;
    DBuf srht_rows, srht_dbits;   // SRHT descriptor (sampled rows, sign bits of D)
    // Signed column sampling: idx, sgn and pos into the handle (the SRHT descriptor's
    // sampler and signs over [0, n)).
    void make_colsample() {
        const int64_t n = P.n, l = P.l;
        DBuf perm(al, (size_t)n * sizeof(int32_t)), D(al, (size_t)n * sizeof(float));
        P.bl_idx.reset(al, (size_t)l * sizeof(int32_t));
        P.bl_sgn.reset(al, (size_t)l * sizeof(double));
        P.bl_pos.reset(al, (size_t)n * sizeof(int32_t));
        launch_srht_prepare(n, l, P.opts.seed, n, perm.as<int32_t>(), P.bl_idx.as<int32_t>(), D.as<float>(), st);
        launch_colsample_prep(n, l, D.as<float>(), P.bl_idx.as<int32_t>(), P.bl_sgn.as<double>(),
                              P.bl_pos.as<int32_t>(), st);
        check_launch();
    }

    void make_omega() {
        const int64_t n = P.n, l = P.l;
        const rr_build_opts& o = P.opts;
        const bool kernel = is_kernel(P.op);
        const bool f32path = o.prec != RR_PREC_FP64;
        P.omega_dt = f32path ? DT_F32 : DT_F64;
        const size_t oes = P.omega_dt == DT_F32 ? sizeof(float) : sizeof(double);
        P.Omega.reset(al, (size_t)n * l * oes);
        const bool bf16_omega = (kernel && f32path) || (!kernel && o.prec == RR_PREC_MIXED);
        ldo = (n + 7) / 8 * 8;
        if (bf16_omega) {
            // padding rows [n, ldo) stay zero: the bf16 MFMA sketches read whole 8-row chunks
            ob_buf.reset(al, (size_t)ldo * l * 2);
            RR_HIP(hipMemsetAsync(ob_buf.ptr(), 0, (size_t)ldo * l * 2, st));
        }
        void* gen = bf16_omega ? ob_buf.ptr() : P.Omega.ptr();
        const int gdt = bf16_omega ? DT_BF16 : P.omega_dt;
        const int64_t gld = bf16_omega ? ldo : n;
        if (o.sketch == RR_SK_GAUSSIAN) {
            launch_gauss_fill(gen, gdt, n, l, gld, o.seed, st);
        } else if (o.sketch == RR_SK_COLSAMPLE) {
            make_colsample();
            launch_colsample_fill(gdt, n, l, gld, P.bl_idx.as<int32_t>(), P.bl_sgn.as<double>(), gen, st);
        } else {
            int64_t s = 1;
            while (s < n) s *= 2;
            DBuf perm(al, (size_t)s * sizeof(int32_t)), D(al, (size_t)n * sizeof(float));
            srht_rows.reset(al, (size_t)l * sizeof(int32_t));
            launch_srht_prepare(n, l, o.seed, s, perm.as<int32_t>(), srht_rows.as<int32_t>(), D.as<float>(), st);
            launch_srht_fill(gen, gdt, n, l, gld, D.as<float>(), srht_rows.as<int32_t>(), st);
            if (kernel && f32path) {   // the kernel sketch generates this Omega itself
                srht_dbits.reset(al, (size_t)((n + 31) / 32) * sizeof(uint32_t));
                launch_srht_dbits(n, D.as<float>(), srht_dbits.as<uint32_t>(), st);
            }
        }
        if (bf16_omega) launch_copy_mat(DT_BF16, ob_buf.ptr(), ldo, P.omega_dt, P.Omega.ptr(), n, n, l, st);
        Ob = ob_buf.ptr();
        check_launch();
    }

    // q = 1 (eq. testmatrix): Omega <- A X for the X just drawn, stored the way
    // make_omega stores a test matrix (bf16-rounded where the sketch reads bf16).
    void apply_power(const void* A16) {
        if (P.opts.power_q != 1) return;
        const int64_t n = P.n, l = P.l;
        const bool bf16_omega = ob_buf.ptr() != nullptr;
        const int ydt = bf16_omega ? DT_F32 : DT_F64;
        DBuf Y0 = mat(n, l, ydt == DT_F32 ? sizeof(float) : sizeof(double));
        sketch(P.Omega.ptr(), P.omega_dt, 0.0, Y0.ptr(), ydt, A16);
        srht_dbits.release();   // Omega is no longer the SRHT: the sketch reads it
        srht_rows.release();
        if (bf16_omega) {
            launch_copy_mat(DT_F32, Y0.ptr(), n, DT_BF16, ob_buf.ptr(), ldo, n, l, st);
            launch_copy_mat(DT_BF16, ob_buf.ptr(), ldo, P.omega_dt, P.Omega.ptr(), n, n, l, st);
        } else {
            launch_copy_mat(DT_F64, Y0.ptr(), n, P.omega_dt, P.Omega.ptr(), n, n, l, st);
        }
        check_launch();
    }

    // Y = A Omega + mu Omega (the sketch, q = 0).
    void sketch(const void* Om, int odt, double mu, void* Y, int ydt, const void* A16) {
        const int64_t n = P.n, l = P.l;
        if (is_kernel(P.op)) {
            const KernelOp k = kernel_op_of(P);
            if (ydt == DT_F32) {
                DBuf ws(al, (kernel_sketch_ws_floats(n, l) + 1) * sizeof(float));
                launch_kernel_gemm_bf16x2(k, Ob, ldo, l, mu, (float*)Y, n, ws.as<float>(), st,
                                          srht_dbits.ptr() ? srht_rows.as<int32_t>() : nullptr,
                                          srht_dbits.as<uint32_t>());
            } else {
                launch_kernel_gemm_f64(k, (const double*)Om, n, l, mu, (double*)Y, n, st);
            }
            check_launch();
            return;
        }
        if (A16 && ydt == DT_F32) {   // mixed precision: bf16 MFMA, float32 Y
            launch_dense_gemm_bf16(n, l, A16, n, Ob, ldo, mu, (float*)Y, n, st);
            check_launch();
            return;
        }
        launch_copy_mat(odt, Om, n, DT_F64, Y, n, n, l, st);
        launch_scale_mat((double*)Y, n, n, l, mu, st);
        if (A16) gemm(DT_BF16, false, odt, false, n, l, n, A16, n, Om, n, (double*)Y, n, 1.0, 1.0);
        else if (P.A32.ptr()) gemm(DT_F32, false, odt, false, n, l, n, P.A32.ptr(), n, Om, n, (double*)Y, n, 1.0, 1.0);
        else gemm(DT_F64, false, odt, false, n, l, n, P.op.A, P.op.lda, Om, n, (double*)Y, n, 1.0, 1.0);
        check_launch();
    }

    // Q (n x k) R (k x k) = Y (n x k).  Sketched: Algorithm prec_chol_qr with the
    // sparse sign embedding Theta (2k x n, stream theta_seed); plain: Algorithm
    // chol_qr.  The block products read Y row-major in float64 (Yt, made here;
    // handed back through yt_out when asked for): a row of Y is what Theta adds,
    // and float64 operands keep the float64 MFMA GEMM at full load width.
    // side(yt), when given, is called once Y^T is queued, to start work that needs
    // only Y (it may queue on the second stream).
    template <typename Side>
    void orth(const void* Y, int ydt, int64_t k, uint64_t theta_seed, double* Q, double* R,
              DBuf* yt_out, Side&& side) {
        const int64_t n = P.n;
        DBuf Yt = mat(k, n);   // column-major k x n = Y^T
        launch_transpose_f64(ydt, n, k, Y, n, Yt.as<double>(), k, st);
        const double* yt = Yt.as<double>();
        side(yt);
        if (P.opts.orth == RR_ORTH_SKETCHED_CHOLQR) {
            DBuf S = mat(2 * k, k);
            launch_theta_apply(n, k, theta_seed, yt, k, S.as<double>(), 2 * k, st);
            DBuf Rsk = mat(k, k);
            const size_t hwd = householder_ws_doubles(2 * k, k);
            DBuf hws(al, hwd * sizeof(double));
            launch_householder_r(S.as<double>(), 2 * k, k, 2 * k, Rsk.as<double>(), k, hws.as<double>(),
                                 hwd, st);
            hws.release();
            S.release();
            check_launch();
            DBuf Rskinv = mat(k, k);
            launch_tri_inv_upper(Rsk.as<double>(), k, k, Rskinv.as<double>(), k, st);
            DBuf W = mat(n, k);
            gemm_upper_b(true, n, k, k, yt, k, Rskinv.as<double>(), k, W.as<double>(), n);
            DBuf GW = mat(k, k);
            gram(k, n, W.as<double>(), n, GW.as<double>(), k);
            chol_ladder(GW.as<double>(), k);            // GW <- R_chol
            DBuf Rcinv = mat(k, k);
            launch_tri_inv_upper(GW.as<double>(), k, k, Rcinv.as<double>(), k, st);
            gemm_upper_b(false, n, k, k, W.as<double>(), n, Rcinv.as<double>(), k, Q, n);
            gemm(DT_F64, false, DT_F64, false, k, k, k, GW.ptr(), k, Rsk.ptr(), k, R, k);  // R = R_chol R_sk
            launch_zero_lower(R, k, k, st);
        } else {
            gemm(DT_F64, false, DT_F64, true, k, k, n, yt, k, yt, k, R, k);
            launch_symmetrize(R, k, k, st);
            chol_ladder(R, k);
            DBuf Rinv = mat(k, k);
            launch_tri_inv_upper(R, k, k, Rinv.as<double>(), k, st);
            gemm_upper_b(true, n, k, k, yt, k, Rinv.as<double>(), k, Q, n);
        }
        check_launch();
        if (yt_out) *yt_out = std::move(Yt);
    }
    void orth(const void* Y, int ydt, int64_t k, uint64_t theta_seed, double* Q, double* R) {
        orth(Y, ydt, k, theta_seed, Q, R, nullptr, [](const double*) {});
    }

    // Power iteration: v <- op(v)/||op(v)|| from a Gaussian start (stream seed);
    // returns ||op(v)|| for the last unit v.
    template <typename Op>
    double power_norm(Op op, uint64_t seed, int iters) {
        const int64_t n = P.n;
        DBuf v(al, n * sizeof(double)), w(al, n * sizeof(double));
        launch_gauss_fill(v.ptr(), DT_F64, n, 1, n, seed, st);
        launch_dot_part(n, v.as<double>(), v.as<double>(), vparts.as<double>(), st);
        launch_normalize(n, v.as<double>(), v.as<double>(), vparts.as<double>(), vec_blocks(n), scal.as<double>() + 1, st);
        for (int it = 0; it < iters; ++it) {
            op(v.as<double>(), w.as<double>());
            launch_dot_part(n, w.as<double>(), w.as<double>(), vparts.as<double>(), st);
            launch_normalize(n, v.as<double>(), w.as<double>(), vparts.as<double>(), vec_blocks(n), scal.as<double>(), st);
        }
        check_launch();
        double lam = 0.0;
        RR_HIP(hipMemcpyAsync(&lam, scal.ptr(), sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        return lam;
    }

    // lambda_max of a small spd k x k matrix on the device: Lanczos with full
    // reorthogonalisation run until its Ritz residual bound is below 1e-14 lambda
    // (k <= lanczos_max_dim()), else 200 power-iteration steps.
    double small_lambda_max(const double* G, int64_t k, uint64_t seed) {
        if (k <= lanczos_max_dim()) {
            DBuf ws(al, lanczos_ws_doubles(k) * sizeof(double));
            double* o3 = scal.as<double>() + 8;
            launch_lanczos_lmax(G, k, k, seed, ws.as<double>(), o3, st);
            check_launch();
            double h[3] = {0.0, 0.0, 0.0};
            RR_HIP(hipMemcpyAsync(h, o3, sizeof(h), hipMemcpyDeviceToHost, st));
            sync();
            return h[0];
        }
        DBuf v(al, k * sizeof(double)), w(al, k * sizeof(double));
        launch_gauss_fill(v.ptr(), DT_F64, k, 1, k, seed, st);
        launch_dot_part(k, v.as<double>(), v.as<double>(), vparts.as<double>(), st);
        launch_normalize(k, v.as<double>(), v.as<double>(), vparts.as<double>(), vec_blocks(k), scal.as<double>() + 1, st);
        for (int it = 0; it < 200; ++it) {
            gemm(DT_F64, false, DT_F64, false, k, 1, k, G, k, v.ptr(), k, w.as<double>(), k);
            launch_dot_part(k, w.as<double>(), w.as<double>(), vparts.as<double>(), st);
            launch_normalize(k, v.as<double>(), w.as<double>(), vparts.as<double>(), vec_blocks(k), scal.as<double>(), st);
        }
        check_launch();
        double lam = 0.0;
        RR_HIP(hipMemcpyAsync(&lam, scal.ptr(), sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        return lam;
    }

    // Basis-less C-RandRAND (Algorithm BL_RandRAND_PCG steps 1-3) for a kernel
    // operator and a signed column-sampling Omega: Y = A_mu Omega streams through
    // row blocks (never stored whole) to form S = Theta Y and Y^T Y; R from the Q-less
    // preconditioned Cholesky QR (Algorithm prec_chol_qr) or Cholesky QR; Q^T Q =
    // R^{-T} Y^T Y R^{-1} gives T, Omega^T A_mu Omega gives G, and the power iterations
    // apply Q through Y and R.  The apply core is Kr = R^{-1} K R^{-T} over Y.
    void build_basisless(PerMu& pm) {
        const int64_t n = P.n, l = P.l;
        const KernelOp k = kernel_op_of(P);
        const bool f64 = P.opts.prec == RR_PREC_FP64;
        const double mu = pm.mu;
        const int32_t* idx = P.bl_idx.as<int32_t>();
        const double* sgn = P.bl_sgn.as<double>();
        const int32_t* pos = P.bl_pos.as<int32_t>();
        const int64_t rb = std::max<int64_t>(256, std::min<int64_t>(n, ((int64_t)1 << 22) / l));
        DBuf Yb = mat(rb, l), GY = mat(l, l), S = mat(2 * l, l);
        const bool sketched = P.opts.orth == RR_ORTH_SKETCHED_CHOLQR;
        for (int64_t r0 = 0; r0 < n; r0 += rb) {
            const int64_t rows = std::min(rb, n - r0);
            launch_kblock_y(k, f64, idx, sgn, l, mu, r0, rows, nullptr, nullptr, Yb.as<double>(), l, st);
            if (sketched)
                launch_theta_apply_rows(rows, r0, l, P.opts.seed + 1, Yb.as<double>(), l, S.as<double>(), 2 * l,
                                        r0 > 0, st);
            // Yb (row-major rows x l) is the column-major l x rows matrix Y_b^T
            gemm(DT_F64, false, DT_F64, true, l, l, rows, Yb.ptr(), l, Yb.ptr(), l, GY.as<double>(), l, 1.0,
                 r0 > 0 ? 1.0 : 0.0);
        }
        Yb.release();
        launch_symmetrize(GY.as<double>(), l, l, st);
        pm.R.reset(al, (size_t)l * l * sizeof(double));
        if (sketched) {
            DBuf Rsk = mat(l, l), Rski = mat(l, l), tmp = mat(l, l), W = mat(l, l);
            const size_t hwd = householder_ws_doubles(2 * l, l);
            DBuf hws(al, hwd * sizeof(double));
            launch_householder_r(S.as<double>(), 2 * l, l, 2 * l, Rsk.as<double>(), l, hws.as<double>(), hwd, st);
            launch_tri_inv_upper(Rsk.as<double>(), l, l, Rski.as<double>(), l, st);
            gemm(DT_F64, true, DT_F64, false, l, l, l, Rski.ptr(), l, GY.ptr(), l, tmp.as<double>(), l);
            gemm(DT_F64, false, DT_F64, false, l, l, l, tmp.ptr(), l, Rski.ptr(), l, W.as<double>(), l);
            launch_symmetrize(W.as<double>(), l, l, st);
            chol_ladder(W.as<double>(), l);   // W <- R_chol
            gemm(DT_F64, false, DT_F64, false, l, l, l, W.ptr(), l, Rsk.ptr(), l, pm.R.as<double>(), l);
            launch_zero_lower(pm.R.as<double>(), l, l, st);
        } else {
            launch_copy_mat(DT_F64, GY.ptr(), l, DT_F64, pm.R.ptr(), l, l, l, st);
            chol_ladder(pm.R.as<double>(), l);
        }
        S.release();
        DBuf Rinv = mat(l, l), tmp = mat(l, l);
        launch_tri_inv_upper(pm.R.as<double>(), l, l, Rinv.as<double>(), l, st);
        // T = 2I - R^{-T} Y^T Y R^{-1}
        pm.T.reset(al, (size_t)l * l * sizeof(double));
        gemm(DT_F64, true, DT_F64, false, l, l, l, Rinv.ptr(), l, GY.ptr(), l, tmp.as<double>(), l);
        gemm(DT_F64, false, DT_F64, false, l, l, l, tmp.ptr(), l, Rinv.ptr(), l, pm.T.as<double>(), l);
        launch_symmetrize(pm.T.as<double>(), l, l, st);
        orth_error(pm.T.as<double>(), l);
        launch_two_minus(pm.T.as<double>(), l, l, st);
        // G from C = Omega^T A_mu Omega (sampled rows and columns of A_mu, signed)
        DBuf C = mat(l, l);
        launch_kblock_y(k, f64, idx, sgn, l, mu, 0, l, idx, sgn, C.as<double>(), l, st);
        pm.G.reset(al, (size_t)l * l * sizeof(double));
        core_G(C.as<double>(), pm.R.as<double>(), pm.G.as<double>(), l);
        DBuf TG = mat(l, l), TGT = mat(l, l);
        gemm(DT_F64, false, DT_F64, false, l, l, l, pm.T.ptr(), l, pm.G.ptr(), l, TG.as<double>(), l);
        gemm(DT_F64, false, DT_F64, false, l, l, l, TG.ptr(), l, pm.T.ptr(), l, TGT.as<double>(), l);
        launch_symmetrize(TGT.as<double>(), l, l, st);
        // cores over Y: X -> R^{-1} X R^{-T}
        auto over_y = [&](const double* X, double* outm, bool sym) {
            gemm(DT_F64, false, DT_F64, false, l, l, l, Rinv.ptr(), l, X, l, tmp.as<double>(), l);
            gemm(DT_F64, false, DT_F64, true, l, l, l, tmp.ptr(), l, Rinv.ptr(), l, outm, l);
            if (sym) launch_symmetrize(outm, l, l, st);
        };
        DBuf KPi = mat(l, l), KnegPi = mat(l, l), KPt = mat(l, l);
        over_y(pm.T.as<double>(), KPi.as<double>(), true);
        launch_axpby_mat(-1.0, KPi.as<double>(), l, 0.0, KPi.as<double>(), l, KnegPi.as<double>(), l, l, l, st);
        over_y(TGT.as<double>(), KPt.as<double>(), true);
        DBuf cv(al, (size_t)l * sizeof(double)), dv(al, (size_t)l * sizeof(double));
        DBuf t1(al, (size_t)n * sizeof(double)), t2(al, (size_t)n * sizeof(double));
        DBuf opp(al, ((size_t)operator_part_count(P) + 1) * sizeof(double));
        // out = rcoef v + Y Kcore Y^T v (Kcore symmetric)
        auto proj = [&](const double* Kcore, const double* v, double rcoef, double* out) {
            launch_kblock_rows(k, f64, idx, sgn, l, v, mu, cv.as<double>(), nullptr, st);
            launch_core_apply(l, Kcore, l, cv.as<double>(), 1, dv.as<double>(), nullptr, st);
            launch_kblock_cols(k, f64, idx, sgn, pos, l, dv.as<double>(), mu, v, rcoef, out, nullptr, nullptr, st);
        };
        auto amu = [&](const double* v, double* out) {
            apply_operator(P, v, mu, out, opp.as<double>(), kws.as<double>(), false, nullptr, st);
        };
        if (P.opts.tau_rule == RR_TAU_NYS) {
            pm.tau = 1.0 / small_lambda_max(pm.G.as<double>(), l, P.opts.seed + 3);
            pm.normE = pm.lam = std::nan("");
        } else {
            // ||E||: v -> (I-Pi) A_mu (I-Pi) v;  lam: v -> Pi A_mu Pi~ v
            pm.normE = power_norm([&](const double* v, double* w) {
                proj(KnegPi.as<double>(), v, 1.0, t1.as<double>());
                amu(t1.as<double>(), t2.as<double>());
                proj(KnegPi.as<double>(), t2.as<double>(), 1.0, w);
            }, P.opts.seed + 2, P.opts.power_iters);
            pm.lam = power_norm([&](const double* v, double* w) {
                proj(KPt.as<double>(), v, 0.0, t1.as<double>());
                amu(t1.as<double>(), t2.as<double>());
                proj(KPi.as<double>(), t2.as<double>(), 0.0, w);
            }, P.opts.seed + 3, P.opts.power_iters);
            if (!std::isfinite(pm.normE) || !(pm.lam > 0.0) || !std::isfinite(pm.lam))
                throw RrError{RR_ENOTSPD, "power-iteration estimates of ||E|| or lam are not positive"};
            if (!(pm.normE > 0.0)) pm.tau = 1.0 / small_lambda_max(pm.G.as<double>(), l, P.opts.seed + 3);
            else if (P.opts.tau_rule == RR_TAU_OPT && mu > 0.0) pm.tau = std::sqrt(mu * pm.normE / pm.lam);
            else pm.tau = P.opts.rho * pm.normE / pm.lam;
        }
        // K = tau T G T - T (or the re-orthogonalised tau T G - T); the solve's core apply
        // computes Kc^T c, so Kc = (R^{-1} K R^{-T})^T = R^{-1} K^T R^{-T}
        DBuf Kt = mat(l, l);
        if (P.opts.reorth) {
            DBuf GT = mat(l, l);
            gemm(DT_F64, false, DT_F64, false, l, l, l, pm.G.ptr(), l, pm.T.ptr(), l, GT.as<double>(), l);
            launch_axpby_mat(pm.tau, GT.as<double>(), l, -1.0, pm.T.as<double>(), l, Kt.as<double>(), l, l, l, st);
        } else {
            launch_axpby_mat(pm.tau, TGT.as<double>(), l, -1.0, pm.T.as<double>(), l, Kt.as<double>(), l, l, l, st);
        }
        pm.Kc.reset(al, (size_t)l * l * sizeof(double));
        over_y(Kt.as<double>(), pm.Kc.as<double>(), !P.opts.reorth);
        check_launch();
    }

    // tau and its estimates for one shift; cores are kb x kb over the basis Qb.
    // M: Qb^T Qb (kb x kb), for the merged projections below.
    void tau_for(PerMu& pm, const double* negT, const double* TGT, const double* T, const double* G,
                 int64_t l, const double* M) {
        const int64_t n = P.n;
        const double mu = pm.mu;
        if (P.opts.tau_rule == RR_TAU_NYS) {
            const double lmax = small_lambda_max(G, l, P.opts.seed + 3);
            pm.tau = 1.0 / lmax;
            pm.normE = std::nan("");
            pm.lam = std::nan("");
            return;
        }
        // The two power iterations run side by side so each step costs one
        // two-column operator pass (every kernel entry evaluated once):
        //   ||E||: v <- (I-Pi) A_mu (I-Pi) v,   lam: v <- Pi A_mu Pi~ v,
        // with Pi = Qb T Qb^T and Pi~ = Qb TGT Qb^T.  The output projection of a step
        // and the input projection of the next are one projection, since scaling
        // commutes with them:
        //   (I-Pi)(I-Pi) = I - Qb (2T - T M T) Qb^T,   Pi~ Pi = Qb (TGT M T) Qb^T,
        // and the norms the steps normalise by come along: ||(I-Pi) y||^2 is
        // y^T (I-Pi)^2 y, the dot the projection kernel forms anyway, and
        // ||Pi y||^2 = c^T (T M T) c with c = Qb^T y.  So a step costs one operator
        // pass and one projection pair instead of two.
        // They only estimate two scalars to a few digits, so a float32-mode
        // kernel operator may add its products in float32 here.
        const int64_t kb = P.kb;
        DBuf U(al, 2 * n * sizeof(double)), Yv(al, 2 * n * sizeof(double));
        DBuf V(al, 2 * n * sizeof(double)), Wv(al, 2 * n * sizeof(double));
        const int nch = gemv_t_chunks(n, kb);
        DBuf cpart(al, (size_t)2 * nch * kb * sizeof(double)), d(al, 3 * kb * sizeof(double));
        DBuf rz(al, (size_t)2 * qd_blocks(n) * sizeof(double));
        DBuf op_part(al, (size_t)2 * operator_part_count(P) * sizeof(double));
        DBuf c1(al, kb * sizeof(double));
        // merged cores: KE = T M T - 2T (with r added back: I - Qb (2T - TMT) Qb^T),
        // KL = TGT M T, B1 = T M T
        DBuf MT = mat(kb, kb), B1 = mat(kb, kb), KE = mat(kb, kb), KL = mat(kb, kb);
        gemm(DT_F64, false, DT_F64, false, kb, kb, kb, M, kb, T, kb, MT.as<double>(), kb);
        gemm(DT_F64, false, DT_F64, false, kb, kb, kb, T, kb, MT.ptr(), kb, B1.as<double>(), kb);
        launch_symmetrize(B1.as<double>(), kb, kb, st);
        launch_axpby_mat(1.0, B1.as<double>(), kb, -2.0, T, kb, KE.as<double>(), kb, kb, kb, st);
        gemm(DT_F64, false, DT_F64, false, kb, kb, kb, TGT, kb, MT.ptr(), kb, KL.as<double>(), kb);
        double* u0 = U.as<double>();
        double* u1 = u0 + n;
        double* y0 = Yv.as<double>();
        double* v0 = V.as<double>();
        double* v1 = v0 + n;
        double* w0 = Wv.as<double>();
        double* w1 = w0 + n;
        double* lam_dev = scal.as<double>();   // [0] ||E||, [1] lam, [2..3] start norms
        launch_gauss_fill(v0, DT_F64, n, 1, n, P.opts.seed + 2, st);
        launch_gauss_fill(v1, DT_F64, n, 1, n, P.opts.seed + 3, st);
        launch_dot_part(n, v0, v0, vparts.as<double>(), st);
        launch_normalize(n, v0, v0, vparts.as<double>(), vec_blocks(n), lam_dev + 2, st);
        launch_dot_part(n, v1, v1, vparts.as<double>(), st);
        launch_normalize(n, v1, v1, vparts.as<double>(), vec_blocks(n), lam_dev + 3, st);
        double* cp = cpart.as<double>();
        double* dd = d.as<double>();
        double* rzp = rz.as<double>();
        // u = [(I-Pi) v0, Pi~ v1]
        apply_projected_pair(P, negT, TGT, v0, 1.0, 0.0, u0, cp, dd, rzp, st);
        for (int it = 0; it < P.opts.power_iters; ++it) {
            apply_operator_multi(P, u0, 2, mu, y0, op_part.as<double>(), kws.as<double>(), false, st,
                                 true);
            // w = [(I-Pi)^2 y0, Pi~ Pi y1] (unnormalised next inputs), y0^T w0 in rzp,
            // c1 = Qb^T y1 and T M T c1 for ||Pi y1||^2
            launch_gemv_t_multi(2, n, kb, P.Qb.as<double>(), n, y0, n, cp, nch, nullptr, st);
            launch_core_apply_triple(kb, KE.as<double>(), KL.as<double>(), B1.as<double>(), kb, cp, nch, dd,
                                     c1.as<double>(), st);
            launch_qd_multi(2, n, kb, P.Qb.as<double>(), n, dd, y0, n, 1.0, 0.0, w0, rzp, nullptr, st);
            launch_normalize_pair(n, u0, w0, rzp, qd_blocks(n), lam_dev + 0, u1, w1, c1.as<double>(),
                                  dd + 2 * kb, kb, lam_dev + 1, st);
        }
        check_launch();
        double lams[2] = {0.0, 0.0};
        RR_HIP(hipMemcpyAsync(lams, lam_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        pm.normE = lams[0];
        pm.lam = lams[1];
        if (!std::isfinite(pm.normE) || !(pm.lam > 0.0) || !std::isfinite(pm.lam))
            throw RrError{RR_ENOTSPD, "power-iteration estimates of ||E|| or lam are not positive"};
        if (!(pm.normE > 0.0)) {
            // range(Q) is the whole space (E = 0): tau from eq. nys_tau keeps P spd
            pm.tau = 1.0 / small_lambda_max(G, l, P.opts.seed + 3);
            return;
        }
        if (P.opts.tau_rule == RR_TAU_OPT && mu > 0.0) pm.tau = std::sqrt(mu * pm.normE / pm.lam);
        else pm.tau = P.opts.rho * pm.normE / pm.lam;
    }

    // G from C = Omega^T Y_mu (l x l) and R:  R_Omega = chol(sym C), H = R_Omega R^{-1}, G = H^T H.
    void core_G(double* C, const double* R, double* G, int64_t l) {
        launch_symmetrize(C, l, l, st);
        chol_ladder(C, l);
        DBuf Rinv = mat(l, l), H = mat(l, l);
        core_G_factored(C, R, G, l, Rinv.as<double>(), H.as<double>(), st, gws.as<double>());
    }
    // the same once C holds R_Omega, on stream s with GEMM workspace ws (gwsd doubles);
    // Rinv and H are l x l scratch
    void core_G_factored(const double* C, const double* R, double* G, int64_t l, double* Rinv, double* H,
                         hipStream_t s, double* ws) {
        launch_tri_inv_upper(R, l, l, Rinv, l, s);
        launch_gemm(DT_F64, false, DT_F64, false, l, l, l, C, l, Rinv, l, H, l, 1.0, 0.0, ws, gwsd, s);
        launch_gemm(DT_F64, true, DT_F64, false, l, l, l, H, l, H, l, G, l, 1.0, 0.0, ws, gwsd, s);
        launch_symmetrize(G, l, l, s);
    }

    // max |Q^T Q - I| into a device word; read after the build's final synchronisation
    DBuf oerr;
    void orth_error(const double* QtQ, int64_t k) {
        if (!oerr.ptr()) oerr.reset(al, sizeof(double));
        launch_max_abs_minus_identity(QtQ, k, k, oerr.as<double>(), st);
    }
};

}  // namespace

extern "C" rr_status rr_build_precond(const rr_operator* A, const double* mus, int32_t n_mu,
                                      const rr_build_opts* opts_in, const rr_allocator* alloc,
                                      void* hip_stream, rr_precond** out) {
    if (out) *out = nullptr;
    return guarded([&]() -> rr_status {
        RR_REQUIRE(out != nullptr, "out is null");
        validate_operator(A);
        RR_REQUIRE(mus != nullptr, "mus is null");
        RR_REQUIRE(n_mu >= 1 && n_mu <= 64, "n_mu must be in [1, 64]");
        for (int i = 0; i < n_mu; ++i)
            RR_REQUIRE(std::isfinite(mus[i]) && mus[i] >= 0.0, "every mu must be finite and >= 0");
        rr_build_opts o;
        if (opts_in) o = *opts_in; else rr_build_opts_default(&o);
        const int64_t n = A->n;
        RR_REQUIRE(o.l >= 0 && o.l <= n, "l must be in [0, n]");
        RR_REQUIRE(o.sketch == RR_SK_GAUSSIAN || o.sketch == RR_SK_SRHT || o.sketch == RR_SK_COLSAMPLE,
                   "unknown sketch");
        RR_REQUIRE(o.orth == RR_ORTH_SKETCHED_CHOLQR || o.orth == RR_ORTH_CHOLQR, "unknown orth");
        RR_REQUIRE(o.basis == RR_BASIS_EXPLICIT || o.basis == RR_BASIS_LESS, "unknown basis");
        RR_REQUIRE(o.reorth == 0 || o.reorth == 1, "reorth must be 0 or 1");
        if (o.basis == RR_BASIS_LESS && o.l > 0) {
            RR_REQUIRE(is_kernel(*A), "a basis-less handle needs a kernel operator");
            RR_REQUIRE(o.sketch == RR_SK_COLSAMPLE, "a basis-less handle needs the COLSAMPLE test matrix");
            RR_REQUIRE(n_mu == 1, "a basis-less handle holds one shift");
            RR_REQUIRE(o.power_q == 0, "a basis-less handle uses q = 0");
        }
        if (o.reorth) RR_REQUIRE(n_mu == 1, "the re-orthogonalised core is built for one shift");
        RR_REQUIRE(o.prec >= RR_PREC_FP64 && o.prec <= RR_PREC_MIXED, "unknown precision");
        RR_REQUIRE(o.tau_rule >= RR_TAU_OPT && o.tau_rule <= RR_TAU_NYS, "unknown tau rule");
        RR_REQUIRE(std::isfinite(o.rho) && o.rho > 0.0, "rho must be finite and > 0");
        RR_REQUIRE(o.power_iters >= 1 && o.power_iters <= 10000, "power_iters must be in [1, 10000]");
        RR_REQUIRE(o.power_q == 0 || o.power_q == 1, "power_q must be 0 or 1");
        RR_REQUIRE(o.multi_shift == RR_MULTI_JOINT || o.multi_shift == RR_MULTI_SHIFTED_CHOL, "unknown multi_shift");
        RR_REQUIRE(o.l_max >= 0 && o.l_max <= n, "l_max must be in [0, n]");
        if (o.l_max > o.l) {
            RR_REQUIRE(o.l >= 1 && n_mu == 1, "adaptive l needs l >= 1 and a single shift");
            RR_REQUIRE(o.tau_rule != RR_TAU_NYS, "adaptive l needs the ||E|| estimate (tau rule OPT or RHO)");
            RR_REQUIRE(std::isfinite(o.ad_factor) && o.ad_factor > 0.0, "ad_factor must be > 0");
        }
        if (n_mu > 1 && o.l > 0) RR_REQUIRE(2 * o.l <= n, "several shifts need 2l <= n (joint basis)");
        if (alloc) RR_REQUIRE(alloc->alloc && alloc->free, "allocator callbacks are null");
        require_device();
        if (o.l_max > o.l) {
            // adaptive sketch size (eq. ad_criterion, with ||E|| for ||(I-Pi) A_mu||)
            const double t_all = now_ms();
            const double thr = o.ad_factor * std::pow((double)n / (double)o.l_max, 1.0 / (2.0 * o.power_q + 2.0)) *
                               std::fabs(mus[0]);
            rr_build_opts oi = o;
            oi.l_max = 0;
            double prev = -1.0;
            while (true) {
                rr_precond* h = nullptr;
                const rr_status s1 = rr_build_precond(A, mus, 1, &oi, alloc, hip_stream, &h);
                if (s1 != RR_OK) return s1;
                const double nE = h->per[0].normE;
                const bool done = nE <= thr || oi.l >= o.l_max || (prev >= 0.0 && nE > 0.9 * prev);
                if (done) {
                    h->ms_build = now_ms() - t_all;
                    h->opts.l_max = o.l_max;
                    *out = h;
                    return RR_OK;
                }
                prev = nE;
                rr_precond_destroy(h);
                oi.l = std::min<int64_t>(2 * oi.l, o.l_max);
            }
        }

        const double t0 = now_ms();
        hipStream_t st = (hipStream_t)hip_stream;
        std::unique_ptr<rr_precond> H(new rr_precond());
        rr_precond& P = *H;
        P.op = *A;
        P.opts = o;
        P.n = n;
        P.l = o.l;
        P.joint = (n_mu > 1 && o.l > 0);
        P.kb = P.joint ? 2 * o.l : o.l;
        P.alloc.st = st;
        if (alloc) { P.alloc.a = *alloc; P.alloc.custom = true; }
        RR_HIP(hipGetDevice(&P.device));
        const Alloc* al = &P.alloc;

        // A0: operator setup
        setup_operator(P, st);
        P.per.resize(n_mu);
        for (int i = 0; i < n_mu; ++i) P.per[i].mu = mus[i];
        if (o.l == 0) {
            RR_HIP(hipGetLastError());
            RR_HIP(hipStreamSynchronize(st));
            P.ms_build = now_ms() - t0;
            *out = H.release();
            return RR_OK;
        }

        Builder B(P, st);
        const int64_t l = o.l;
        if (o.basis == RR_BASIS_LESS) {
            P.basisless = true;
            B.make_colsample();
            B.build_basisless(P.per[0]);
            RR_HIP(hipGetLastError());
            if (B.oerr.ptr())
                RR_HIP(hipMemcpyAsync(&P.orth_err, B.oerr.ptr(), sizeof(double), hipMemcpyDeviceToHost, st));
            RR_HIP(hipStreamSynchronize(st));
            P.ms_build = now_ms() - t0;
            *out = H.release();
            return RR_OK;
        }
        // A1: Omega
        B.make_omega();
        const bool kernel = is_kernel(*A);
        const bool f32path = o.prec != RR_PREC_FP64;

        // bf16 copy of a dense A for the mixed-precision sketch (freed after it)
        DBuf A16;
        if (o.prec == RR_PREC_MIXED && !kernel) {
            A16.reset(al, (size_t)n * n * 2);
            launch_copy_mat(DT_F64, A->A, A->lda, DT_BF16, A16.ptr(), n, n, n, st);
        }
        B.apply_power(A16.ptr());
        const int ydt = ((kernel && f32path) || (!kernel && o.prec == RR_PREC_MIXED)) ? DT_F32 : DT_F64;
        const size_t yes = ydt == DT_F32 ? sizeof(float) : sizeof(double);
        P.Qb.reset(al, (size_t)n * P.kb * sizeof(double));

        if (!P.joint) {
            PerMu& pm = P.per[0];
            const double mu = pm.mu;
            // A2: sketch
            DBuf Y = B.mat(n, l, yes);
            B.sketch(P.Omega.ptr(), P.omega_dt, mu, Y.ptr(), ydt, A16.ptr());
            A16.release();
            // A3: orthogonalisation
            pm.R.reset(al, (size_t)l * l * sizeof(double));
            // A4's C = Omega^T Y and its Cholesky R_Omega need only Y: they run on a
            // second stream beside the orthogonalisation (C^T = Y^T Omega with
            // float64 operands; C is symmetrised before it is factored).
            // Buffers the second stream touches are allocated on the main stream before
            // it is ordered after the main stream, and freed only after the join (or,
            // on an error, after the guard below has waited for the second stream).
            DBuf Yt, C = B.mat(l, l), Ccopy = B.mat(l, l), Od;
            // An SRHT Omega (still the SRHT: q = 0) gives C^T = Y^T Omega by chunked
            // Walsh-Hadamard transforms of the columns of Y instead of a GEMM against a
            // float64 copy of Omega: far fewer flops and bytes beside the orthogonalisation.
            int64_t hs = 1;
            while (hs < n) hs *= 2;
            const bool fwht = B.srht_dbits.ptr() && B.srht_rows.ptr();
            if (fwht) Od = B.mat(srht_yt_omega_ws_doubles(n, l, hs), 1);
            else if (P.omega_dt != DT_F64) Od = B.mat(n, l);
            struct SideGuard {
                Builder& b;
                ~SideGuard() {
                    if (b.st2) (void)hipStreamSynchronize(b.st2);
                }
            } side_guard{B};
            auto side = [&](const double* yt) {
                B.side_begin();
                if (fwht) {
                    launch_srht_yt_omega(ydt, n, l, hs, Y.ptr(), n, B.srht_dbits.as<uint32_t>(),
                                         B.srht_rows.as<int32_t>(), Od.as<double>(), C.as<double>(), l, B.st2);
                    launch_symmetrize(C.as<double>(), l, l, B.st2);
                    B.chol_start(C.as<double>(), l, Ccopy.as<double>(), B.st2, B.status2.as<int32_t>(),
                                 B.gws2.as<double>(), B.gwsd);
                    return;
                }
                const void* om = P.Omega.ptr();
                if (P.omega_dt != DT_F64) {
                    launch_copy_mat(P.omega_dt, P.Omega.ptr(), n, DT_F64, Od.ptr(), n, n, l, B.st2);
                    om = Od.ptr();
                }
                launch_gemm(DT_F64, false, DT_F64, false, l, l, n, yt, l, om, n, C.as<double>(), l, 1.0, 0.0,
                            B.gws2.as<double>(), B.gwsd, B.st2);
                launch_symmetrize(C.as<double>(), l, l, B.st2);
                B.chol_start(C.as<double>(), l, Ccopy.as<double>(), B.st2, B.status2.as<int32_t>(),
                             B.gws2.as<double>(), B.gwsd);
            };
            B.orth(Y.ptr(), ydt, l, o.seed + 1, P.Qb.as<double>(), pm.R.as<double>(), &Yt, side);
            B.chol_finish(C.as<double>(), l, Ccopy.as<double>(), B.st2, B.status2.as<int32_t>(),
                          B.gws2.as<double>(), B.gwsd);
            B.side_join();
            Y.release();
            Yt.release();
            Od.release();
            Ccopy.release();
            // A4: core, refined projector, tau, apply core.  G (from R and R_Omega) on
            // the second stream while the main one forms T = 2I - Q^T Q.
            pm.G.reset(al, (size_t)l * l * sizeof(double));
            DBuf Rinv = B.mat(l, l), H = B.mat(l, l);
            SideGuard side_guard2{B};   // freed after the second stream is idle
            B.side_begin();
            B.core_G_factored(C.as<double>(), pm.R.as<double>(), pm.G.as<double>(), l, Rinv.as<double>(),
                              H.as<double>(), B.st2, B.gws2.as<double>());
            pm.T.reset(al, (size_t)l * l * sizeof(double));
            B.gram(l, n, P.Qb.as<double>(), n, pm.T.as<double>(), l);
            B.orth_error(pm.T.as<double>(), l);
            launch_two_minus(pm.T.as<double>(), l, l, st);
            B.side_join();
            DBuf TG = B.mat(l, l), TGT = B.mat(l, l), negT = B.mat(l, l);
            B.gemm(DT_F64, false, DT_F64, false, l, l, l, pm.T.ptr(), l, pm.G.ptr(), l, TG.as<double>(), l);
            B.gemm(DT_F64, false, DT_F64, false, l, l, l, TG.ptr(), l, pm.T.ptr(), l, TGT.as<double>(), l);
            launch_symmetrize(TGT.as<double>(), l, l, st);
            launch_axpby_mat(-1.0, pm.T.as<double>(), l, 0.0, pm.T.as<double>(), l, negT.as<double>(), l, l, l, st);
            {
                DBuf M = B.mat(l, l);   // Q^T Q = 2I - T
                launch_axpby_mat(-1.0, pm.T.as<double>(), l, 0.0, pm.T.as<double>(), l, M.as<double>(), l, l, l, st);
                launch_add_diag(M.as<double>(), l, l, 2.0, st);
                B.tau_for(pm, negT.as<double>(), TGT.as<double>(), pm.T.as<double>(), pm.G.as<double>(), l,
                          M.as<double>());
            }
            pm.Kc.reset(al, (size_t)l * l * sizeof(double));
            if (o.reorth) {
                // eq. c_randrand_reorth: K = tau T G - T; the core apply computes Kc^T c,
                // so Kc = K^T = tau G T - T
                DBuf GT = B.mat(l, l);
                B.gemm(DT_F64, false, DT_F64, false, l, l, l, pm.G.ptr(), l, pm.T.ptr(), l, GT.as<double>(), l);
                launch_axpby_mat(pm.tau, GT.as<double>(), l, -1.0, pm.T.as<double>(), l, pm.Kc.as<double>(), l, l, l, st);
            } else {
                launch_axpby_mat(pm.tau, TGT.as<double>(), l, -1.0, pm.T.as<double>(), l, pm.Kc.as<double>(), l, l, l,
                                 st);
            }
            B.check_launch();
        } else {
            // several shifts (Section 5.1): the apply basis Qb (n x 2l) and, per shift,
            // Qred (2l x l) with Q_mu = Qb Qred and R with A_mu Omega = Q_mu R.
            // JOINT: Qb = orth([Omega, A Omega]); Qred, R = qr(Qb^T A Omega + mu Qb^T Omega).
            // SHIFTED_CHOL: A_alpha Omega = Q_a R_a at alpha = max mu, Qb = [Q_a, Omega R_a^{-1}],
            // R_chol = chol(W2 + 2 (mu - alpha) W1 + (mu - alpha)^2 W0), Qred = [I; (mu - alpha) I]
            // R_chol^{-1}, R = R_chol R_a.
            const int64_t k2 = 2 * l;
            const bool shifted = o.multi_shift == RR_MULTI_SHIFTED_CHOL;
            double alpha = 0.0;
            for (int im = 0; im < n_mu; ++im) alpha = std::max(alpha, P.per[im].mu);
            DBuf Y0 = B.mat(n, l, yes);
            B.sketch(P.Omega.ptr(), P.omega_dt, shifted ? alpha : 0.0, Y0.ptr(), ydt, A16.ptr());
            A16.release();
            double* Qj = P.Qb.as<double>();
            DBuf Zj, Oj, OAO = B.mat(l, l), OO = B.mat(l, l), QQ = B.mat(k2, k2);
            DBuf Ra, W2, W1, W0;
            B.gemm(P.omega_dt, true, ydt, false, l, l, n, P.Omega.ptr(), n, Y0.ptr(), n, OAO.as<double>(), l);
            B.gemm(P.omega_dt, true, P.omega_dt, false, l, l, n, P.Omega.ptr(), n, P.Omega.ptr(), n, OO.as<double>(), l);
            if (!shifted) {
                DBuf Z = B.mat(n, k2);
                launch_copy_mat(P.omega_dt, P.Omega.ptr(), n, DT_F64, Z.ptr(), n, n, l, st);
                launch_copy_mat(ydt, Y0.ptr(), n, DT_F64, Z.as<double>() + (size_t)n * l, n, n, l, st);
                DBuf Rj = B.mat(k2, k2);
                B.orth(Z.ptr(), DT_F64, k2, o.seed + 1, Qj, Rj.as<double>());
                Z.release();
                Zj = B.mat(k2, l);
                Oj = B.mat(k2, l);
                B.gemm(DT_F64, true, ydt, false, k2, l, n, Qj, n, Y0.ptr(), n, Zj.as<double>(), k2);
                B.gemm(DT_F64, true, P.omega_dt, false, k2, l, n, Qj, n, P.Omega.ptr(), n, Oj.as<double>(), k2);
                B.gram(k2, n, Qj, n, QQ.as<double>(), k2);
                B.orth_error(QQ.as<double>(), k2);
            } else {
                Ra = B.mat(l, l);
                B.orth(Y0.ptr(), ydt, l, o.seed + 1, Qj, Ra.as<double>());
                DBuf Rai = B.mat(l, l), tmp = B.mat(l, l);
                launch_tri_inv_upper(Ra.as<double>(), l, l, Rai.as<double>(), l, st);
                double* Oma = Qj + (size_t)n * l;
                B.gemm(P.omega_dt, false, DT_F64, false, n, l, l, P.Omega.ptr(), n, Rai.ptr(), l, Oma, n);
                B.gram(k2, n, Qj, n, QQ.as<double>(), k2);
                W2 = B.mat(l, l);
                W0 = B.mat(l, l);
                W1 = B.mat(l, l);
                launch_copy_mat(DT_F64, QQ.ptr(), k2, DT_F64, W2.ptr(), l, l, l, st);
                launch_copy_mat(DT_F64, QQ.as<double>() + (size_t)l * k2 + l, k2, DT_F64, W0.ptr(), l, l, l, st);
                // W1 = R_a^{-T} (Omega^T A_alpha Omega) R_a^{-1}; OAO holds Omega^T A_alpha Omega here
                B.gemm(DT_F64, true, DT_F64, false, l, l, l, Rai.ptr(), l, OAO.ptr(), l, tmp.as<double>(), l);
                B.gemm(DT_F64, false, DT_F64, false, l, l, l, tmp.ptr(), l, Rai.ptr(), l, W1.as<double>(), l);
                launch_symmetrize(W1.as<double>(), l, l, st);
                // OAO <- Omega^T A Omega = Omega^T A_alpha Omega - alpha Omega^T Omega
                launch_axpby_mat(1.0, OAO.as<double>(), l, -alpha, OO.as<double>(), l, OAO.as<double>(), l, l, l, st);
            }
            Y0.release();
            const size_t hwd = std::max<size_t>((size_t)k2 * l + l + 16, householder_ws_doubles(k2, l));
            DBuf hws(al, hwd * sizeof(double));
            for (int im = 0; im < n_mu; ++im) {
                PerMu& pm = P.per[im];
                const double mu = pm.mu;
                pm.Qred.reset(al, (size_t)k2 * l * sizeof(double));
                pm.R.reset(al, (size_t)l * l * sizeof(double));
                if (!shifted) {
                    DBuf Mred = B.mat(k2, l);
                    launch_axpby_mat(1.0, Zj.as<double>(), k2, mu, Oj.as<double>(), k2, Mred.as<double>(), k2, k2, l, st);
                    launch_householder_qr(Mred.as<double>(), k2, l, k2, pm.Qred.as<double>(), k2, pm.R.as<double>(), l,
                                          hws.as<double>(), hwd, st);
                } else {
                    const double sft = mu - alpha;
                    DBuf Wm = B.mat(l, l), Rci = B.mat(l, l);
                    launch_axpby_mat(1.0, W2.as<double>(), l, 2.0 * sft, W1.as<double>(), l, Wm.as<double>(), l, l, l, st);
                    launch_axpby_mat(1.0, Wm.as<double>(), l, sft * sft, W0.as<double>(), l, Wm.as<double>(), l, l, l, st);
                    launch_symmetrize(Wm.as<double>(), l, l, st);
                    B.chol_ladder(Wm.as<double>(), l);   // Wm <- R_chol
                    launch_tri_inv_upper(Wm.as<double>(), l, l, Rci.as<double>(), l, st);
                    launch_copy_mat(DT_F64, Rci.ptr(), l, DT_F64, pm.Qred.ptr(), k2, l, l, st);
                    launch_axpby_mat(sft, Rci.as<double>(), l, 0.0, Rci.as<double>(), l, pm.Qred.as<double>() + l, k2,
                                     l, l, st);
                    B.gemm(DT_F64, false, DT_F64, false, l, l, l, Wm.ptr(), l, Ra.ptr(), l, pm.R.as<double>(), l);
                    launch_zero_lower(pm.R.as<double>(), l, l, st);
                }
                B.check_launch();
                DBuf C = B.mat(l, l);
                launch_axpby_mat(1.0, OAO.as<double>(), l, mu, OO.as<double>(), l, C.as<double>(), l, l, l, st);
                pm.G.reset(al, (size_t)l * l * sizeof(double));
                B.core_G(C.as<double>(), pm.R.as<double>(), pm.G.as<double>(), l);
                // T = 2I - Qred^T (Qb^T Qb) Qred
                DBuf tmp = B.mat(k2, l);
                B.gemm(DT_F64, false, DT_F64, false, k2, l, k2, QQ.ptr(), k2, pm.Qred.ptr(), k2, tmp.as<double>(), k2);
                pm.T.reset(al, (size_t)l * l * sizeof(double));
                B.gemm(DT_F64, true, DT_F64, false, l, l, k2, pm.Qred.ptr(), k2, tmp.ptr(), k2, pm.T.as<double>(), l);
                launch_symmetrize(pm.T.as<double>(), l, l, st);
                if (shifted) B.orth_error(pm.T.as<double>(), l);   // Q_mu^T Q_mu against I
                launch_two_minus(pm.T.as<double>(), l, l, st);
                DBuf TG = B.mat(l, l), TGT = B.mat(l, l);
                B.gemm(DT_F64, false, DT_F64, false, l, l, l, pm.T.ptr(), l, pm.G.ptr(), l, TG.as<double>(), l);
                B.gemm(DT_F64, false, DT_F64, false, l, l, l, TG.ptr(), l, pm.T.ptr(), l, TGT.as<double>(), l);
                launch_symmetrize(TGT.as<double>(), l, l, st);
                // lift l x l cores to the 2l-dimensional basis coordinates: X -> Qred X Qred^T
                auto lift = [&](const double* X, double* outm) {
                    DBuf t1 = B.mat(k2, l);
                    B.gemm(DT_F64, false, DT_F64, false, k2, l, l, pm.Qred.ptr(), k2, X, l, t1.as<double>(), k2);
                    B.gemm(DT_F64, false, DT_F64, true, k2, k2, l, t1.ptr(), k2, pm.Qred.ptr(), k2, outm, k2);
                    launch_symmetrize(outm, k2, k2, st);
                };
                DBuf Tt = B.mat(k2, k2), TGTt = B.mat(k2, k2), negTt = B.mat(k2, k2);
                lift(pm.T.as<double>(), Tt.as<double>());
                lift(TGT.as<double>(), TGTt.as<double>());
                launch_axpby_mat(-1.0, Tt.as<double>(), k2, 0.0, Tt.as<double>(), k2, negTt.as<double>(), k2, k2, k2, st);
                B.tau_for(pm, negTt.as<double>(), TGTt.as<double>(), Tt.as<double>(), pm.G.as<double>(), l,
                          QQ.as<double>());
                DBuf K = B.mat(l, l);
                launch_axpby_mat(pm.tau, TGT.as<double>(), l, -1.0, pm.T.as<double>(), l, K.as<double>(), l, l, l, st);
                pm.Kc.reset(al, (size_t)k2 * k2 * sizeof(double));
                lift(K.as<double>(), pm.Kc.as<double>());
                B.check_launch();
            }
        }
        RR_HIP(hipGetLastError());
        if (B.oerr.ptr())
            RR_HIP(hipMemcpyAsync(&P.orth_err, B.oerr.ptr(), sizeof(double), hipMemcpyDeviceToHost, st));
        RR_HIP(hipStreamSynchronize(st));
        P.ms_build = now_ms() - t0;
        *out = H.release();
        return RR_OK;
    });
}

// The sketch step alone, for inspection: Y = A Omega + mu Omega exactly as
// rr_build_precond computes it with the same options.
extern "C" rr_status rr_sketch_apply(const rr_operator* A, double mu, const rr_build_opts* opts,
                               double* Y_out, void* hip_stream) {
    return guarded([&]() -> rr_status {
        validate_operator(A);
        RR_REQUIRE(opts != nullptr && Y_out != nullptr, "opts or Y_out is null");
        RR_REQUIRE(std::isfinite(mu) && mu >= 0.0, "mu must be finite and >= 0");
        RR_REQUIRE(opts->l >= 1 && opts->l <= A->n, "l must be in [1, n]");
        RR_REQUIRE(opts->sketch == RR_SK_GAUSSIAN || opts->sketch == RR_SK_SRHT, "unknown sketch");
        RR_REQUIRE(opts->prec >= RR_PREC_FP64 && opts->prec <= RR_PREC_MIXED, "unknown precision");
        require_device();
        hipStream_t st = (hipStream_t)hip_stream;
        rr_precond P;
        P.op = *A;
        P.opts = *opts;
        P.n = A->n;
        P.l = opts->l;
        P.kb = P.l;
        P.alloc.st = st;
        RR_HIP(hipGetDevice(&P.device));
        const int64_t n = P.n, l = P.l;
        const bool kernel = is_kernel(*A);
        setup_operator(P, st);
        Builder B(P, st);
        B.make_omega();
        DBuf A16;
        if (opts->prec == RR_PREC_MIXED && !kernel) {
            A16.reset(&P.alloc, (size_t)n * n * 2);
            launch_copy_mat(DT_F64, A->A, A->lda, DT_BF16, A16.ptr(), n, n, n, st);
        }
        B.apply_power(A16.ptr());
        const int ydt = ((kernel && opts->prec != RR_PREC_FP64) || (!kernel && opts->prec == RR_PREC_MIXED))
                            ? DT_F32 : DT_F64;
        DBuf Y = B.mat(n, l, ydt == DT_F32 ? sizeof(float) : sizeof(double));
        B.sketch(P.Omega.ptr(), P.omega_dt, mu, Y.ptr(), ydt, A16.ptr());
        launch_copy_mat(ydt, Y.ptr(), n, DT_F64, Y_out, n, n, l, st);
        RR_HIP(hipGetLastError());
        RR_HIP(hipStreamSynchronize(st));
        return RR_OK;
    });
}

// Inspection: the build's Cholesky with its shift ladder on a caller matrix.
extern "C" rr_status rr_cholesky_ladder(const double* W, int64_t k, double* R, double* alpha_host,
                                        void* hip_stream) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(W != nullptr && R != nullptr, "W or R is null");
        RR_REQUIRE(k >= 1 && k <= 16384, "k must be in [1, 16384]");
        require_device();
        hipStream_t st = (hipStream_t)hip_stream;
        rr_precond P;
        P.op.kind = RR_OP_DENSE;
        P.n = k;
        P.l = k;
        P.kb = k;
        P.alloc.st = st;
        Builder B(P, st);
        RR_HIP(hipMemcpyAsync(R, W, (size_t)k * k * sizeof(double), hipMemcpyDeviceToDevice, st));
        launch_symmetrize(R, k, k, st);
        const double a = B.chol_ladder(R, k);
        if (alpha_host) *alpha_host = a;
        RR_HIP(hipStreamSynchronize(st));
        return RR_OK;
    });
}

// Inspection: lambda_max of a symmetric psd matrix exactly as the NYS tau rule takes it.
extern "C" rr_status rr_lambda_max(const double* G, int64_t k, uint64_t seed, double* out_host,
                                   void* hip_stream) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(G != nullptr && out_host != nullptr, "G or out is null");
        RR_REQUIRE(k >= 1 && k <= lanczos_max_dim(), "k must be in [1, 1536]");
        require_device();
        hipStream_t st = (hipStream_t)hip_stream;
        Alloc al;
        al.st = st;
        DBuf ws(&al, lanczos_ws_doubles(k) * sizeof(double)), o3(&al, 4 * sizeof(double));
        launch_lanczos_lmax(G, k, k, seed, ws.as<double>(), o3.as<double>(), st);
        RR_HIP(hipGetLastError());
        RR_HIP(hipMemcpyAsync(out_host, o3.ptr(), 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        RR_HIP(hipStreamSynchronize(st));
        return RR_OK;
    });
}
