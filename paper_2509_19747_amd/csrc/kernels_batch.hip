// Kernels of the batched solve: many independent PCG recurrences (one per
// column, each with its own shift mu_j) advanced by fused launches.
//
//  * k_kgemm_f32_mfma : W = scale * K P + diag(mu_col) P for m columns at once in
//      the working precision: float32 entries (the formula of the vector-ALU
//      symmetric matvec over the padded point records) times P in float32 on
//      v_mfma_f32_32x32x2_f32, float32 sums over runs of 64 points added in float64.
//  * k_kgemm_f64_mfma : the same product with float64 entries (the table exp2 of
//      the float64 symmetric matvec) on v_mfma_f64_16x16x4_f64 (float64 mode and
//      the refinement residuals).
//  * per-column dot partials, scalar steps and vector updates with a per-column
//      run flag: converged or restarting columns are left untouched.
#include "common.hpp"
#include "group.hpp"
#include "kentry.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace rr {

typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int KD_BM = 256, KD_BN = 128, KD_BK = 16, KD_THREADS = 1024;

// Block: 16 waves in a 4 (rows) x 4 (columns) grid of 64 x 32 wave tiles (4 x 2
// MFMA tiles, 32 float64 accumulators per lane), four waves per SIMD: the float64
// MFMA pipe needs several resident waves to stay busy.  Per step of 16 points the
// block forms the 256 x 16 kernel tile (thread: one row, 4 points whose records
// arrive through scalar loads; float64 entries: difference form, float64 exp) into
// LDS (k-major) and stages the 16 x 128 slice of P.
template <int KIND, int DM>
__global__ __launch_bounds__(KD_THREADS) void k_kgemm_f64_mfma(
    int64_t n, const float* __restrict__ xa, double g, double kconst, double scale,
    const double* __restrict__ mucol, const double* __restrict__ P, int64_t ldp, int64_t m,
    double* __restrict__ W, int64_t ldw) {
    __shared__ double As[KD_BK][KD_BM + 2];
    __shared__ double Bs[KD_BK][KD_BN + 2];
    __shared__ double tab[EXP2_TAB];
    exp2_table_fill(tab);
    __syncthreads();
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave & 3, wn = wave >> 2;
    const int64_t i0 = (int64_t)blockIdx.x * KD_BM;
    const int64_t c0 = (int64_t)blockIdx.y * KD_BN;

    const int trow = t & (KD_BM - 1);
    const int pg = __builtin_amdgcn_readfirstlane(t >> 8);   // 0..3: which 4 of the 16 points
    const int64_t gi = i0 + trow;
    const int64_t gic = gi < n ? gi : n - 1;
    float xi[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k) xi[k] = xa[gic * DM + k];
    f64x4 acc[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4{0.0, 0.0, 0.0, 0.0};

    // the next step's point records (wave-uniform) and P values are loaded while the
    // current step's MFMAs run
    float xj[4][DM];
    double pv[2];
    auto load = [&](int64_t j0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t gj = j0 + pg * 4 + e;
            const int64_t gjc = gj < n ? gj : n - 1;
#pragma unroll
            for (int k = 0; k < DM; ++k) xj[e][k] = xa[gjc * DM + k];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int64_t gj = j0 + (t & 15), gc = c0 + (t >> 4) + 64 * s;
            pv[s] = (gj < n && gc < m) ? P[gj + gc * ldp] : 0.0;
        }
    };
    load(0);
    for (int64_t j0 = 0; j0 < n; j0 += KD_BK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int p = pg * 4 + e;
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                const double df = (double)xi[k] - (double)xj[e][k];
                r2 = fma(df, df, r2);
            }
            // 2^t with t = -g r^2 / 2 (the float64 entry of the symmetric matvec)
            As[p][trow] = (j0 + p < n) ? kentry64<KIND>(-0.5 * g * r2, kconst, tab) : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) Bs[t & 15][(t >> 4) + 64 * s] = pv[s];
        if (j0 + KD_BK < n) load(j0 + KD_BK);
        __syncthreads();
#pragma unroll
        for (int kc = 0; kc < KD_BK; kc += 4) {
            double a[4], b[2];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = As[kc + (lane >> 4)][wm * 64 + u * 16 + (lane & 15)];
#pragma unroll
            for (int v = 0; v < 2; ++v) b[v] = Bs[kc + (lane >> 4)][wn * 32 + v * 16 + (lane & 15)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[v], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int64_t gc = c0 + wn * 32 + v * 16 + (lane & 15);
            if (gc >= m) continue;
            const double mu = mucol[gc];
            // v_mfma_f64_16x16x4_f64 result layout: element e of lane l is row 4*e + l/16,
            // column l%16 (unlike the f32 16x16x4 form, whose rows are 4*(l/16) + e)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gr = i0 + wm * 64 + u * 16 + 4 * e + (lane >> 4);
                if (gr < n) W[gr + gc * ldw] = fma(scale, acc[u][v][e], mu * P[gr + gc * ldp]);
            }
        }
    }
}

// The working-precision product (float32 and mixed modes): the same float32 entries
// times P rounded to float32 on v_mfma_f32_32x32x2_f32 (twice the float64 MFMA rate),
// with the float32 accumulators added into float64 sums every KF_FLUSH slices of 16
// points, so the sums stay float64 beyond 64-term runs (the float32 working operator
// of the multi-RHS block).  Block: 16 waves in a 4 x 4 grid of 32 x 32 wave tiles
// (one MFMA tile each: 16 float32 and 16 float64 accumulators per lane), a 128 x 16
// kernel tile formed per slice (thread: one row, two points) and a 16 x 128 slice of P.
constexpr int KF32_BM = 128, KF32_BN = 128, KF32_BK = 16, KF32_FLUSH = 4, KF32_THREADS = 1024;
typedef float f32x16_mm __attribute__((ext_vector_type(16)));

template <int KIND, int DM>
__global__ __launch_bounds__(KF32_THREADS) void k_kgemm_f32_mfma(
    int64_t n, const float* __restrict__ xa, const float* __restrict__ sqn, float c, double scale,
    const double* __restrict__ mucol, const double* __restrict__ P, int64_t ldp, int64_t m,
    double* __restrict__ W, int64_t ldw) {
    __shared__ float As[KF32_BK][KF32_BM + 4];
    __shared__ float Bs[KF32_BK][KF32_BN + 4];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave & 3, wn = wave >> 2;
    const int64_t i0 = (int64_t)blockIdx.x * KF32_BM;
    const int64_t c0 = (int64_t)blockIdx.y * KF32_BN;

    const int trow = t & (KF32_BM - 1);
    const int pg = __builtin_amdgcn_readfirstlane(t >> 7);   // 0..7: points 2 pg, 2 pg + 1 of a slice
    const int64_t gi = i0 + trow;
    const int64_t gic = gi < n ? gi : n - 1;
    float xi[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k) xi[k] = xa[gic * DM + k];
    const float mhn = -0.5f * sqn[gic];

    f32x16_mm acc;
    double acc64[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        acc[e] = 0.0f;
        acc64[e] = 0.0;
    }
    // the next slice's point records (wave-uniform) and P values are loaded while the
    // current slice's MFMAs run
    float xj[2][DM], sqj[2];
    double pv[2];
    auto load = [&](int64_t j0) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t gj = j0 + 2 * pg + e;
            const int64_t gjc = gj < n ? gj : n - 1;
#pragma unroll
            for (int k = 0; k < DM; ++k) xj[e][k] = xa[gjc * DM + k];
            sqj[e] = sqn[gjc];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int64_t gj = j0 + (t & 15), gc = c0 + (t >> 4) + 64 * s;
            pv[s] = (gj < n && gc < m) ? P[gj + gc * ldp] : 0.0;
        }
    };
    load(0);
    int slices = 0;
    for (int64_t j0 = 0; j0 < n; j0 += KF32_BK) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int p = 2 * pg + e;
            float sv = kpair_init(mhn, sqj[e]);
#pragma unroll
            for (int k = 0; k < DM; ++k) sv = fmaf(xi[k], xj[e][k], sv);
            As[p][trow] = j0 + p < n ? kval32<KIND>(sv, c) : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) Bs[t & 15][(t >> 4) + 64 * s] = (float)pv[s];
        if (j0 + KF32_BK < n) load(j0 + KF32_BK);
        __syncthreads();
#pragma unroll
        for (int kc = 0; kc < KF32_BK; kc += 2) {
            const float a = As[kc + (lane >> 5)][wm * 32 + (lane & 31)];
            const float b = Bs[kc + (lane >> 5)][wn * 32 + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
        if (++slices == KF32_FLUSH) {
            slices = 0;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                acc64[e] += (double)acc[e];
                acc[e] = 0.0f;
            }
        }
    }
    // accumulator element e of lane l: row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
    const int64_t gc = c0 + wn * 32 + (lane & 31);
    if (gc >= m) return;
    const double mu = mucol[gc];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const double v = acc64[e] + (double)acc[e];
        const int64_t gr = i0 + wm * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (gr < n) W[gr + gc * ldw] = fma(scale, v, mu * P[gr + gc * ldp]);
    }
}

template <int KIND>
static void kd_dispatch(const KernelOp& op, float c, const double* mucol, const double* P,
                        int64_t ldp, int64_t m, double* W, int64_t ldw, hipStream_t st) {
    dim3 grid((unsigned)((op.n + KD_BM - 1) / KD_BM), (unsigned)((m + KD_BN - 1) / KD_BN));
    const double g = kernel_g64(op.kind, op.kconst);
#define KDL(DD) k_kgemm_f64_mfma<KIND, DD><<<grid, KD_THREADS, 0, st>>>(op.n, op.xa, g, op.kconst, op.scale, mucol, P, ldp, m, W, ldw)
    switch (op.dm) {
        case 4: KDL(4); break;
        case 8: KDL(8); break;
        case 16: KDL(16); break;
        default: KDL(32); break;
    }
#undef KDL
}

template <int KIND>
static void kf32_dispatch(const KernelOp& op, float c, const double* mucol, const double* P, int64_t ldp,
                          int64_t m, double* W, int64_t ldw, hipStream_t st) {
    dim3 grid((unsigned)((op.n + KF32_BM - 1) / KF32_BM), (unsigned)((m + KF32_BN - 1) / KF32_BN));
#define KFL(DD) k_kgemm_f32_mfma<KIND, DD><<<grid, KF32_THREADS, 0, st>>>(op.n, op.xa, op.sqn, c, op.scale, mucol, P, ldp, m, W, ldw)
    switch (op.dm) {
        case 4: KFL(4); break;
        case 8: KFL(8); break;
        case 16: KFL(16); break;
        default: KFL(32); break;
    }
#undef KFL
}

void launch_kernel_matmat_f64(const KernelOp& op, bool f64_entries, const double* mucol,
                              const double* P, int64_t ldp, int64_t m, double* W, int64_t ldw,
                              hipStream_t st) {
    const float c = kernel_c32(op.kind, op.kconst);
    ProfScope prof(f64_entries ? -1 : PROF_KERNEL_MATMAT, st);
    if (op.kind == 1) {
        if (f64_entries) kd_dispatch<1>(op, c, mucol, P, ldp, m, W, ldw, st);
        else kf32_dispatch<1>(op, c, mucol, P, ldp, m, W, ldw, st);
    } else {
        if (f64_entries) kd_dispatch<2>(op, c, mucol, P, ldp, m, W, ldw, st);
        else kf32_dispatch<2>(op, c, mucol, P, ldp, m, W, ldw, st);
    }
}

// W[:, j] += mu_j P[:, j] for a dense operator product computed by the GEMM.
__global__ void k_add_shift_cols(int64_t n, int64_t m, const double* __restrict__ mucol,
                                 const double* __restrict__ P, int64_t ldp, double* __restrict__ W,
                                 int64_t ldw) {
    const int64_t total = n * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, j = e / n;
        W[i + j * ldw] = fma(mucol[j], P[i + j * ldp], W[i + j * ldw]);
    }
}
void launch_add_shift_cols(int64_t n, int64_t m, const double* mucol, const double* P, int64_t ldp,
                           double* W, int64_t ldw, hipStream_t st) {
    int64_t g = (n * m + 255) / 256;
    if (g > 65536) g = 65536;
    k_add_shift_cols<<<(int)g, 256, 0, st>>>(n, m, mucol, P, ldp, W, ldw);
}

// =========================================================== per-column CG
constexpr int BC_THREADS = 256;

int coldot_chunks(int64_t n) {
    int64_t c = (n + 8191) / 8192;
    if (c < 1) c = 1;
    if (c > 32) c = 32;
    return (int)c;
}

// part[ch * m + j] = sum_{i in chunk ch} A[i, j] B[i, j]
__global__ __launch_bounds__(BC_THREADS) void k_coldot(int64_t n, int64_t m,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ part, int64_t rpc) {
    __shared__ double sc[BC_THREADS / WAVE];
    const int64_t j = blockIdx.x, ch = blockIdx.y;
    const int64_t ib = ch * rpc;
    const int64_t ie = (ib + rpc < n) ? ib + rpc : n;
    double acc = 0.0;
    for (int64_t i = ib + threadIdx.x; i < ie; i += BC_THREADS) acc = fma(A[i + j * lda], B[i + j * ldb], acc);
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) part[ch * m + j] = acc;
}
void launch_coldot(int64_t n, int64_t m, const double* A, int64_t lda, const double* B, int64_t ldb,
                   double* part, hipStream_t st) {
    const int nch = coldot_chunks(n);
    const int64_t rpc = (n + nch - 1) / nch;
    dim3 grid((unsigned)m, (unsigned)nch);
    k_coldot<<<grid, BC_THREADS, 0, st>>>(n, m, A, lda, B, ldb, part, rpc);
}

RR_DEV double colsum(const ColParts& pt, int64_t j) {
    double s = 0.0;
    for (int c = 0; c < pt.nch; ++c) s += pt.p[(int64_t)c * pt.cs + j * pt.js];
    return s;
}

// start a cycle for the columns flagged in `start`: rho = r^T z, run = 1
__global__ void k_bstate_start(ColParts part, int64_t m, BState* st,
                               const int32_t* __restrict__ start, const double* __restrict__ target2,
                               int32_t maxit) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || !start[j]) return;
    const double rz = colsum(part, j);
    st[j].rho = rz;
    st[j].alpha = st[j].beta = 0.0;
    st[j].target2 = target2[j];
    st[j].maxit = maxit;
    st[j].code = STOP_NONE;
    st[j].run = 1;
    if (!(rz > 0.0) || !isfinite(rz)) { st[j].run = 0; st[j].code = STOP_BREAKDOWN; }
}
static int cgrid(int64_t m) { return (int)((m + 255) / 256); }
void launch_bstate_start(ColParts part, int64_t m, BState* st, const int32_t* start,
                         const double* target2, int32_t maxit, hipStream_t s) {
    k_bstate_start<<<cgrid(m), 256, 0, s>>>(part, m, st, start, target2, maxit);
}

// column blocks: grid (row chunks, m); the column's run flag is uniform per block
static dim3 vgrid(int64_t n, int64_t m) {
    int64_t gx = (n + BC_THREADS * 8 - 1) / (BC_THREADS * 8);
    if (gx < 1) gx = 1;
    return dim3((unsigned)gx, (unsigned)m);
}
int bxr_blocks(int64_t n) { return (int)vgrid(n, 1).x; }
// Fused per-column steps.  Every block of column j recomputes the column's scalar
// from the block partials (one block-wide sum in a fixed order, so all blocks get
// the same value), applies its share of the vector update, and the last block of
// the column to finish (a per-column counter; that block resets it to zero)
// records the scalars and the stop tests in the column state.  A column that is
// not running at launch is left alone by every block.
RR_DEV double colsum_block(const ColParts& pt, int64_t j, double* sc) {
    double v = 0.0;
    for (int c = threadIdx.x; c < pt.nch; c += blockDim.x) v += pt.p[(int64_t)c * pt.cs + j * pt.js];
    return block_sum(v, sc);
}
RR_DEV bool last_block_of_column(int32_t* cnt, int64_t j, int nbx, int* flag) {
    __threadfence();   // this block's partials and vector updates are visible device-wide
    if (threadIdx.x == 0) *flag = atomicAdd(&cnt[j], 1) == nbx - 1;
    __syncthreads();
    if (!*flag) return false;
    __threadfence();   // the other blocks' partials are read after this point
    return true;
}

// alpha_j = rho_j / p_j^T w_j; x_j += alpha_j p_j, r_j -= alpha_j w_j, partials of
// ||r_j||^2; last block: pw, alpha, ||r||^2, the iteration count and the stop tests.
// Block bx of the nbx blocks of column j (shared with the grouped serving kernel).
// The column's scalars after its x and r update: pw, alpha, ||r||^2, the iteration
// count and the stop tests (thread 0 of the block that records them).
RR_DEV void bxr_record(int64_t j, BState* st, double pwj, bool ok, double a, double rr) {
    st[j].pw = pwj;
    if (!ok) { st[j].run = 0; st[j].code = STOP_BREAKDOWN; return; }
    st[j].alpha = a;
    st[j].rr = rr;
    const int it = st[j].iters + 1;
    st[j].iters = it;
    if (!isfinite(rr)) { st[j].run = 0; st[j].code = STOP_BREAKDOWN; }
    else if (rr <= st[j].target2) { st[j].run = 0; st[j].code = STOP_TARGET; }
    else if (it >= st[j].maxit) { st[j].run = 0; st[j].code = STOP_MAXIT; }
}

// alpha_j and block bx's share of x_j += alpha_j p_j, r_j -= alpha_j w_j; writes the
// block's partial of ||r_j||^2.  Returns false when the column is not running.
RR_DEV bool bxr_apply(int bx, int nbx, int64_t j, int64_t n, double* __restrict__ X, int64_t ldx,
                      double* __restrict__ R, const double* __restrict__ P, const double* __restrict__ W,
                      const BState* st, const ColParts& pw, double* __restrict__ rr_part, double* sc,
                      double& pwj, bool& ok, double& a) {
    if (!st[j].run) return false;
    pwj = colsum_block(pw, j, sc);
    ok = pwj > 0.0 && isfinite(pwj);
    a = ok ? st[j].rho / pwj : 0.0;
    double acc = 0.0;
    if (ok)
        for (int64_t i = (int64_t)bx * BC_THREADS + threadIdx.x; i < n; i += (int64_t)nbx * BC_THREADS) {
            X[i + j * ldx] = fma(a, P[i + j * n], X[i + j * ldx]);
            const double ri = fma(-a, W[i + j * n], R[i + j * n]);
            R[i + j * n] = ri;
            acc = fma(ri, ri, acc);
        }
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) rr_part[j * nbx + bx] = acc;
    return true;
}

// Fused: the last block of the column to finish records the scalars.
RR_DEV void bxr_block(int bx, int nbx, int64_t j, int64_t n, double* __restrict__ X, int64_t ldx,
                      double* __restrict__ R, const double* __restrict__ P, const double* __restrict__ W,
                      BState* st, const ColParts& pw, double* __restrict__ rr_part, int32_t* cnt) {
    __shared__ double sc[BC_THREADS / WAVE];
    __shared__ int last;
    double pwj, a;
    bool ok;
    if (!bxr_apply(bx, nbx, j, n, X, ldx, R, P, W, st, pw, rr_part, sc, pwj, ok, a)) return;
    if (!last_block_of_column(cnt, j, nbx, &last)) return;
    const double rr = colsum_block(ColParts{rr_part, nbx, 1, (int64_t)nbx}, j, sc);
    if (threadIdx.x != 0) return;
    cnt[j] = 0;
    bxr_record(j, st, pwj, ok, a, rr);
}
__global__ __launch_bounds__(BC_THREADS) void k_bxr_fused(int64_t n, double* __restrict__ X, int64_t ldx,
                                                         double* __restrict__ R, const double* __restrict__ P,
                                                         const double* __restrict__ W, BState* st, ColParts pw,
                                                         double* __restrict__ rr_part, int32_t* cnt) {
    bxr_block(blockIdx.x, gridDim.x, blockIdx.y, n, X, ldx, R, P, W, st, pw, rr_part, cnt);
}

// Split (wide column blocks): the update without the election of a column's last
// block, whose device-scope fence writes back the L2 on every block; one block per
// column then records the scalars from the same fixed-order sums.
__global__ __launch_bounds__(BC_THREADS) void k_bxr_part(int64_t n, double* __restrict__ X, int64_t ldx,
                                                        double* __restrict__ R, const double* __restrict__ P,
                                                        const double* __restrict__ W, const BState* st,
                                                        ColParts pw, double* __restrict__ rr_part) {
    __shared__ double sc[BC_THREADS / WAVE];
    double pwj, a;
    bool ok;
    (void)bxr_apply(blockIdx.x, gridDim.x, blockIdx.y, n, X, ldx, R, P, W, st, pw, rr_part, sc, pwj, ok, a);
}
__global__ __launch_bounds__(BC_THREADS) void k_bxr_tail(int nbx, BState* st, ColParts pw,
                                                        const double* __restrict__ rr_part) {
    __shared__ double sc[BC_THREADS / WAVE];
    const int64_t j = blockIdx.x;
    if (!st[j].run) return;
    const double pwj = colsum_block(pw, j, sc);
    const bool ok = pwj > 0.0 && isfinite(pwj);
    const double a = ok ? st[j].rho / pwj : 0.0;
    const double rr = colsum_block(ColParts{rr_part, nbx, 1, (int64_t)nbx}, j, sc);
    if (threadIdx.x == 0) bxr_record(j, st, pwj, ok, a, rr);
}

// beta_j = r_j^T z_j / rho_j and block bx's share of p_j = z_j + beta_j p_j.
// Returns false when the column is not running.
RR_DEV bool bp_apply(int bx, int nbx, int64_t j, int64_t n, const double* __restrict__ Z,
                     double* __restrict__ P, const BState* st, const ColParts& rz, double* sc, double& rzj,
                     bool& ok, double& b) {
    if (!st[j].run) return false;
    rzj = colsum_block(rz, j, sc);
    ok = rzj > 0.0 && isfinite(rzj);
    b = ok ? rzj / st[j].rho : 0.0;
    if (ok)
        for (int64_t i = (int64_t)bx * BC_THREADS + threadIdx.x; i < n; i += (int64_t)nbx * BC_THREADS)
            P[i + j * n] = fma(b, P[i + j * n], Z[i + j * n]);
    return true;
}
RR_DEV void bp_record(int64_t j, BState* st, double rzj, bool ok, double b) {
    if (!ok) { st[j].run = 0; st[j].code = STOP_BREAKDOWN; return; }
    st[j].beta = b;
    st[j].rho = rzj;
}

// Fused: the last block of the column records beta and rho.
RR_DEV void bp_block(int bx, int nbx, int64_t j, int64_t n, const double* __restrict__ Z,
                     double* __restrict__ P, BState* st, const ColParts& rz, int32_t* cnt) {
    __shared__ double sc[BC_THREADS / WAVE];
    __shared__ int last;
    double rzj, b;
    bool ok;
    if (!bp_apply(bx, nbx, j, n, Z, P, st, rz, sc, rzj, ok, b)) return;
    if (!last_block_of_column(cnt, j, nbx, &last)) return;
    if (threadIdx.x != 0) return;
    cnt[j] = 0;
    bp_record(j, st, rzj, ok, b);
}
__global__ __launch_bounds__(BC_THREADS) void k_bp_fused(int64_t n, const double* __restrict__ Z,
                                                        double* __restrict__ P, BState* st, ColParts rz,
                                                        int32_t* cnt) {
    bp_block(blockIdx.x, gridDim.x, blockIdx.y, n, Z, P, st, rz, cnt);
}
__global__ __launch_bounds__(BC_THREADS) void k_bp_part(int64_t n, const double* __restrict__ Z,
                                                       double* __restrict__ P, const BState* st, ColParts rz) {
    __shared__ double sc[BC_THREADS / WAVE];
    double rzj, b;
    bool ok;
    (void)bp_apply(blockIdx.x, gridDim.x, blockIdx.y, n, Z, P, st, rz, sc, rzj, ok, b);
}
__global__ __launch_bounds__(BC_THREADS) void k_bp_tail(BState* st, ColParts rz) {
    __shared__ double sc[BC_THREADS / WAVE];
    const int64_t j = blockIdx.x;
    if (!st[j].run) return;
    const double rzj = colsum_block(rz, j, sc);
    const bool ok = rzj > 0.0 && isfinite(rzj);
    const double b = ok ? rzj / st[j].rho : 0.0;
    if (threadIdx.x == 0) bp_record(j, st, rzj, ok, b);
}

// Column blocks wider than this take the split updates.
constexpr int64_t BUPDATE_FUSED_MAX = 32;

void launch_bxr_fused(int64_t n, int64_t m, double* X, int64_t ldx, double* R, const double* P,
                      const double* W, BState* st, ColParts pw, double* rr_part, int32_t* cnt, hipStream_t s) {
    if (m > BUPDATE_FUSED_MAX) {
        const dim3 g = vgrid(n, m);
        k_bxr_part<<<g, BC_THREADS, 0, s>>>(n, X, ldx, R, P, W, st, pw, rr_part);
        k_bxr_tail<<<(unsigned)m, BC_THREADS, 0, s>>>((int)g.x, st, pw, rr_part);
        return;
    }
    k_bxr_fused<<<vgrid(n, m), BC_THREADS, 0, s>>>(n, X, ldx, R, P, W, st, pw, rr_part, cnt);
}
void launch_bp_fused(int64_t n, int64_t m, const double* Z, double* P, BState* st, ColParts rz, int32_t* cnt,
                     hipStream_t s) {
    if (m > BUPDATE_FUSED_MAX) {
        k_bp_part<<<vgrid(n, m), BC_THREADS, 0, s>>>(n, Z, P, st, rz);
        k_bp_tail<<<(unsigned)m, BC_THREADS, 0, s>>>(st, rz);
        return;
    }
    k_bp_fused<<<vgrid(n, m), BC_THREADS, 0, s>>>(n, Z, P, st, rz, cnt);
}


// dst[:, di(c)] = src[:, si(c)] for c < ncols, si / di = the index lists or the identity
__global__ __launch_bounds__(BC_THREADS) void k_copy_cols(int64_t n, const int32_t* __restrict__ si,
                                                         const double* __restrict__ src, int64_t lds,
                                                         const int32_t* __restrict__ di, double* __restrict__ dst,
                                                         int64_t ldd) {
    const int64_t c = blockIdx.y;
    const int64_t sc = si ? si[c] : c, dc = di ? di[c] : c;
    for (int64_t i = (int64_t)blockIdx.x * BC_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BC_THREADS)
        dst[i + dc * ldd] = src[i + sc * lds];
}
void launch_copy_cols(int64_t n, int64_t ncols, const int32_t* si, const double* src, int64_t lds,
                      const int32_t* di, double* dst, int64_t ldd, hipStream_t s) {
    if (ncols <= 0) return;
    k_copy_cols<<<vgrid(n, ncols), BC_THREADS, 0, s>>>(n, si, src, lds, di, dst, ldd);
}

// For flagged columns: dst[:, j] = src[:, j]
__global__ __launch_bounds__(BC_THREADS) void k_copy_flagged(int64_t n, const double* __restrict__ src,
                                                            int64_t lds, double* __restrict__ dst,
                                                            int64_t ldd, const int32_t* __restrict__ flag) {
    const int64_t j = blockIdx.y;
    if (!flag[j]) return;
    for (int64_t i = (int64_t)blockIdx.x * BC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BC_THREADS)
        dst[i + j * ldd] = src[i + j * lds];
}
void launch_copy_flagged(int64_t n, int64_t m, const double* src, int64_t lds, double* dst,
                         int64_t ldd, const int32_t* flag, hipStream_t s) {
    k_copy_flagged<<<vgrid(n, m), BC_THREADS, 0, s>>>(n, src, lds, dst, ldd, flag);
}

// R = B - T (all columns), used for true residuals
__global__ __launch_bounds__(BC_THREADS) void k_bresid(int64_t n, const double* __restrict__ B,
                                                      int64_t ldb, const double* __restrict__ T,
                                                      double* __restrict__ Rt) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * BC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BC_THREADS)
        Rt[i + j * n] = B[i + j * ldb] - T[i + j * n];
}
void launch_bresid(int64_t n, int64_t m, const double* B, int64_t ldb, const double* T, double* Rt,
                   hipStream_t s) {
    k_bresid<<<vgrid(n, m), BC_THREADS, 0, s>>>(n, B, ldb, T, Rt);
}

// D[:, j] = Dall[mu_idx[j]][:, j]  (per-column choice among the per-shift cores)
__global__ void k_select_cols(int64_t k, int64_t m, const double* __restrict__ Dall,
                              const int32_t* __restrict__ mu_idx, double* __restrict__ D) {
    const int64_t total = k * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % k, j = e / k;
        D[i + j * k] = Dall[(int64_t)mu_idx[j] * k * m + i + j * k];
    }
}
void launch_select_cols(int64_t k, int64_t m, const double* Dall, const int32_t* mu_idx, double* D,
                        hipStream_t s) {
    int64_t g = (k * m + 255) / 256;
    if (g > 65536) g = 65536;
    k_select_cols<<<(int)g, 256, 0, s>>>(k, m, Dall, mu_idx, D);
}

// ------------------------------------------------------------------ grouped
// The x, r and p updates of many requests in one persistent launch each: work item
// w of the list belongs to the request whose first item is the largest <= w; its
// offset w - w0 is block (w - w0) % nbx of column (w - w0) / nbx, the block that
// k_bxr_fused / k_bp_fused would run.
template <bool BP>
__global__ __launch_bounds__(BC_THREADS) void k_group_vec(const GTable* __restrict__ tab,
                                                          const GVec* __restrict__ units, int32_t* ctr) {
    __shared__ int32_t wsh;
    constexpr int L = BP ? GL_BP : GL_BXR;
    const int32_t off = gu(tab->list[L].off), cnt = gu(tab->list[L].count), total = gu(tab->list[L].total);
    GroupCursor cur(ctr, &wsh);
    while (true) {
        const int32_t w = cur.next();
        if (w >= total) return;
        const int32_t ui = group_find(units, off, off + cnt, w, [](const GVec& g) { return g.w0; });
        const GVec& g = units[ui];
        const int32_t nbx = gu(g.nbx), loc = w - gu(g.w0);
        const int64_t j = loc / nbx;
        const ColParts pt{gu(g.pw.p), gu(g.pw.nch), gu(g.pw.cs), gu(g.pw.js)};
        const ColParts rz{gu(g.rz.p), gu(g.rz.nch), gu(g.rz.cs), gu(g.rz.js)};
        if (BP)
            bp_block(loc % nbx, nbx, j, gu(g.n), gu(g.Z), gu(g.P), gu(g.st), rz, gu(g.cnt) + gu(g.m));
        else
            bxr_block(loc % nbx, nbx, j, gu(g.n), gu(g.X), gu(g.ldx), gu(g.R), gu(g.P), gu(g.W), gu(g.st), pt,
                      gu(g.rr_part), gu(g.cnt));
    }
}

void launch_group_vec(bool bp, int blocks, const GTable* tab, const GVec* vecs, int32_t* ctr, hipStream_t st) {
    if (bp) k_group_vec<true><<<blocks, BC_THREADS, 0, st>>>(tab, vecs, ctr);
    else k_group_vec<false><<<blocks, BC_THREADS, 0, st>>>(tab, vecs, ctr);
}

__global__ void k_group_reset(int32_t* ctr, int ncount) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncount; i += gridDim.x * blockDim.x) ctr[i] = 0;
}
void launch_group_reset(int32_t* ctr, int ncount, hipStream_t st) {
    k_group_reset<<<(ncount + 255) / 256, 256, 0, st>>>(ctr, ncount);
}

}  // namespace rr
