// Column-block products shared by the batched and block solvers: the operator
// product A_mu P for every column (each column under its own shift), the
// C-RandRAND preconditioner P R for every column, GEMMs on the solve stream and
// fixed-order column dots.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.hpp"

namespace rr {

constexpr int64_t KMULTI_MAX = 32;

struct Batch;
// Runs one batch of PCG iterations of a column block elsewhere (the serving loop's
// grouped replays); returns once they have completed on the device.
struct BatchRunner {
    virtual ~BatchRunner() = default;
    virtual rr_status run(Batch& bt, double* X, int64_t ldx) = 0;
};

struct Batch {
    const rr_precond& P;
    hipStream_t st;
    int64_t n, m, kb;
    int64_t mp;           // columns of P, W and their product partials (m, or padded to whole column blocks)
    Alloc alloc;          // the handle's allocator, ordered on the solve stream
    const Alloc* al;
    DBuf R, Pm, Z, W, T, parts, C, Dall, D, state, start, target2, mucol, muidx, gws;
    DBuf cidx, mucomp;    // column list and shifts of a compact restart product
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
    // grouped layout (serving): every column pair and projection group has its own
    // partials, so that all of them can run in one launch
    bool grouped = false;
    DBuf gpart;               // slot partials, gpart_doubles per column (a block at its first column)
    size_t gpart_doubles = 0;
    DBuf gcpart, gdcols;      // Q^T R partials (m x gch x kb) and D (m x kb) per column

    // Width of the grouped kernel product's column block starting at column c0: four
    // columns (the last ones zero padding) while at least three are left and the
    // records allow it, else two or one.
    static int mat_width(int64_t m, int64_t c0, int dm) {
        const int64_t left = m - c0;
        if (left >= 3 && kernel_mma_max_cols(dm) >= 4) return 4;
        return left >= 2 ? 2 : 1;
    }
    static int64_t padded_cols(int64_t m, int dm) {
        int64_t c = 0;
        while (c < m) c += mat_width(m, c, dm);
        return c;
    }

    Batch(const rr_precond& p, hipStream_t s, int64_t mcols, bool grouped_layout = false)
        : P(p), st(s), n(p.n), m(mcols), kb(p.kb),
          mp(grouped_layout && is_kernel(p.op) ? padded_cols(mcols, kernel_record_len(p.op.d)) : mcols),
          alloc(p.alloc), al(&alloc), grouped(grouped_layout) {
        alloc.st = s;
        const size_t nm = (size_t)n * m * sizeof(double), nmp = (size_t)n * mp * sizeof(double);
        R.reset(al, nm); Pm.reset(al, nmp); Z.reset(al, nm); W.reset(al, nmp); T.reset(al, nm);
        if (mp > m) {
            // the padding column of the last pair is zero (and stays so: nothing updates it)
            RR_HIP(hipMemsetAsync(Pm.ptr(), 0, nmp, st));
            RR_HIP(hipMemsetAsync(W.ptr(), 0, nmp, st));
        }
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
        cidx.reset(al, (size_t)m * sizeof(int32_t));
        mucomp.reset(al, (size_t)m * sizeof(double));
        gwsd = std::max<size_t>((size_t)8 * std::max<int64_t>(kb, 1) * m, (size_t)1 << 20);
        gws.reset(al, gwsd * sizeof(double));
        // a few columns: the symmetric matvec kernel (each entry formed once per
        // group of up to 8 columns, float64 sums) beats a 128-column MFMA tile
        kmulti = is_kernel(p.op) && p.opts.prec != RR_PREC_FP64 && m <= KMULTI_MAX;
        if (kmulti) {
            kws.reset(al, (kernel_matvec_ws_doubles(n, p.op.d, (int)std::min<int64_t>(m, 8)) + 1) * sizeof(double));
            kdot.reset(al, (size_t)kernel_matvec_blocks(n) * mp * sizeof(double));
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
        if (group_ok()) {
            gpart_doubles = kernel_mma_ws_doubles(n, 1);
            gpart.reset(al, (size_t)mp * gpart_doubles * sizeof(double));
            gcpart.reset(al, (size_t)m * gch * kb * sizeof(double));
            gdcols.reset(al, (size_t)m * kb * sizeof(double));
        }
    }

    // The grouped iterations cover one shift, the float32-class kernel product on bf16
    // MFMA and the streaming projection (the serving loop's requests); other column
    // blocks run their own iterations.
    bool group_ok() const {
        return grouped && kmulti && single && pmax > 0 && kb > 0 && kernel_mma_ok(n, P.op.d);
    }
    // Width of the projection group starting at column c0 (the same grouping as precond).
    int group_width(int64_t c0) const {
        const int64_t left = m - c0;
        return left >= pmax ? pmax : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    }

    void gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
              const void* B, int64_t ldb, double* Cm, int64_t ldc, double alpha, double beta,
              int dta = DT_F64) {
        launch_gemm(dta, ta, DT_F64, tb, M, N, K, A, lda, B, ldb, Cm, ldc, alpha, beta, gws.as<double>(), gwsd, st);
    }

    // Wout = A_mu Pin for every column (fp64: float64 operator).  Returns the block
    // partials of Pin_j^T Wout_j when the product produced them (nch = 0 otherwise).
    // mc columns (default all m) under the shifts mu_c (default the columns' own).
    ColParts matmat(const double* Pin, int64_t ldp, double* Wout, bool fp64, int64_t mc = -1,
                    const double* mu_c = nullptr) {
        if (mc < 0) mc = m;
        const double* muc = mu_c ? mu_c : mucol.as<double>();
        if (kmulti && fp64 && ldp == n) {
            // a few columns under the float64 operator: the pair-once float64 matvec,
            // two columns per pass
            const KernelOp k = kernel_op_of(P);
            launch_kernel_matvec_multi(k, true, Pin, (int)mc, 0.0, Wout, kdot.as<double>(), kws.as<double>(),
                                       nullptr, st);
            launch_add_shift_cols(n, mc, muc, Pin, ldp, Wout, n, st);
            return ColParts{nullptr, 0, 0, 0};
        }
        if (kmulti && !fp64 && ldp == n) {
            const KernelOp k = kernel_op_of(P);
            const int nblk = kernel_matvec_blocks(n);
            launch_kernel_matvec_multi(k, false, Pin, (int)mc, single ? mu1 : 0.0, Wout, kdot.as<double>(),
                                       kws.as<double>(), nullptr, st);
            if (single) return ColParts{kdot.as<double>(), nblk, 1, nblk};
            launch_add_shift_cols(n, mc, muc, Pin, ldp, Wout, n, st);
            return ColParts{nullptr, 0, 0, 0};
        }
        if (is_kernel(P.op)) {
            const KernelOp k = kernel_op_of(P);
            launch_kernel_matmat_f64(k, fp64 || P.opts.prec == RR_PREC_FP64, muc, Pin, ldp, mc, Wout, n, st);
        } else {
            if (!fp64 && P.A32.ptr()) gemm(false, false, n, mc, n, P.A32.ptr(), n, Pin, ldp, Wout, n, 1.0, 0.0, DT_F32);
            else gemm(false, false, n, mc, n, P.op.A, P.op.lda, Pin, ldp, Wout, n, 1.0, 0.0);
            launch_add_shift_cols(n, mc, muc, Pin, ldp, Wout, n, st);
        }
        return ColParts{nullptr, 0, 0, 0};
    }

    // Tout[:, j] = A_mu(j) X[:, j] for the columns j in cols (a restart's true
    // residuals).  A strict subset goes through the product as a compact block: its
    // columns are gathered into Z, multiplied into W (both are recomputed by the next
    // iteration before use) and scattered into Tout.  hmu: every column's shift.
    void product_cols(const double* X, int64_t ldx, double* Tout, bool fp64, const std::vector<int32_t>& cols,
                      const std::vector<double>& hmu) {
        const int64_t c = (int64_t)cols.size();
        if (c == 0) return;
        if (c == m) {
            matmat(X, ldx, Tout, fp64);
            return;
        }
        std::vector<double> muc((size_t)c);
        for (int64_t q = 0; q < c; ++q) muc[q] = hmu[cols[q]];
        RR_HIP(hipMemcpyAsync(cidx.ptr(), cols.data(), c * sizeof(int32_t), hipMemcpyHostToDevice, st));
        RR_HIP(hipMemcpyAsync(mucomp.ptr(), muc.data(), c * sizeof(double), hipMemcpyHostToDevice, st));
        launch_copy_cols(n, c, cidx.as<int32_t>(), X, ldx, nullptr, Z.as<double>(), n, st);
        matmat(Z.as<double>(), n, W.as<double>(), fp64, c, mucomp.as<double>());
        launch_copy_cols(n, c, nullptr, W.as<double>(), n, cidx.as<int32_t>(), Tout, n, st);
        // the copies read host vectors staged by the runtime; keep them until the work ran
        RR_HIP(hipStreamSynchronize(st));
    }

    // Zout = P_{mu(j)} Rin for every column.  Returns the block partials of
    // Rin_j^T Zout_j when the projection produced them (nch = 0 otherwise).
    ColParts precond(const double* Rin, double* Zout) {
        const double* Qb = P.Qb.as<double>();
        if (pmax > 0) {
            const double* Kc = P.per[mus_used[0]].Kc.as<double>();
            const int nb = qd_blocks(n);
            for (int64_t c0 = 0; c0 < m;) {
                const int nr = group_width(c0);
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


}  // namespace rr
