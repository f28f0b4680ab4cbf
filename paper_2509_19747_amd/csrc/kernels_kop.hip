// Kernel (Gram) operators formed on the fly: A = scale * K(X, X) with the
// Gaussian RBF or Matern-3/2 kernel (kernel ridge regression, Section 7.2.2,
// eq. kernel), reached only through its entries.
//
//  * launch_kernel_matvec(_multi): y = scale*K u + mu u (the PCG matvec).
//      float32 entries: the symmetric kernel of kernels_ksym.hip.
//      float64 entries: k_kmv_f64 below; rows are split over (row block,
//      j slice), each slice writes partial row sums, and a second kernel adds
//      them in a fixed order (deterministic).
//  * the float32-mode sketch A_mu Omega on bf16 MFMA is in kernels_ksketch.hip.
//  * k_kgemm_f64    : float64 vector-ALU variant (float64 mode).
//
// Entry formulas are in kentry.hpp (the float32 entry is bitwise symmetric).
#include "common.hpp"
#include "kentry.hpp"
#include "kernels.hpp"
#include "prof.hpp"

#include <algorithm>

namespace rr {

__global__ void k_sqnorms(const float* __restrict__ pts, int64_t n, int d, float* __restrict__ sqn) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int k = 0; k < d; ++k) {
            const float v = pts[(int64_t)k * n + i];
            s = fmaf(v, v, s);
        }
        sqn[i] = s;
    }
}
void launch_sqnorms(const float* pts, int64_t n, int d, float* sqn, hipStream_t st) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    k_sqnorms<<<(int)g, 256, 0, st>>>(pts, n, d, sqn);
}

int kernel_record_len(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32; }

__global__ void k_point_records(const float* __restrict__ pts, int64_t n, int d, int dm,
                                float* __restrict__ xa) {
    const int64_t total = n * dm;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / dm;
        const int k = (int)(e - i * dm);
        xa[e] = k < d ? pts[(int64_t)k * n + i] : 0.0f;
    }
}
__global__ void k_point_records64(const float* __restrict__ pts, int64_t n, int d, int dm, double g,
                                  double* __restrict__ xd, double* __restrict__ hd) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < dm; ++k) {
            const double v = k < d ? (double)pts[(int64_t)k * n + i] : 0.0;
            xd[i * dm + k] = v;
            s = fma(v, v, s);
        }
        hd[i] = -0.5 * g * s;
    }
}

double kernel_g64(int kind, double kconst) {
    return kind == 1 ? 2.0 * kconst * 1.4426950408889634074 : 1.0;
}

void launch_point_records64(const float* pts, int64_t n, int d, int dm, double g, double* xd, double* hd,
                            hipStream_t st) {
    int64_t gr = (n + 255) / 256;
    if (gr > 65536) gr = 65536;
    k_point_records64<<<(int)gr, 256, 0, st>>>(pts, n, d, dm, g, xd, hd);
}

void launch_point_records(const float* pts, int64_t n, int d, int dm, float* xa, hipStream_t st) {
    int64_t g = (n * dm + 255) / 256;
    if (g > 8192) g = 8192;
    k_point_records<<<(int)g, 256, 0, st>>>(pts, n, d, dm, xa);
}

// ======================================================== kernel matvec
constexpr int KMV_THREADS = 256;

int kernel_matvec_blocks(int64_t n) { return (int)((n + 255) / 256); }

// Stage 1, float64 entries (difference form, float64 exp).
constexpr int KMV64_R = 4;
constexpr int KMV64_ROWS = KMV_THREADS * KMV64_R;
template <int KIND, int NR>
__global__ __launch_bounds__(KMV_THREADS) void k_kmv_f64(int64_t n, int d,
                                                         const float* __restrict__ pts,
                                                         double kconst,
                                                         const double* __restrict__ u,
                                                         double* __restrict__ part,
                                                         int64_t jper,
                                                         const int32_t* __restrict__ stop) {
    if (stop && *stop) return;
    const int64_t rbase = (int64_t)blockIdx.x * KMV64_ROWS + threadIdx.x;
    double xi[KMV64_R][16];
    double acc[KMV64_R][NR];
    const int dl = d < 16 ? d : 16;
#pragma unroll
    for (int r = 0; r < KMV64_R; ++r) {
        const int64_t i = rbase + (int64_t)r * KMV_THREADS;
        const int64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int k = 0; k < 16; ++k) xi[r][k] = (k < dl) ? (double)pts[(int64_t)k * n + ic] : 0.0;
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[r][q] = 0.0;
    }
    const int64_t jb = (int64_t)blockIdx.y * jper;
    const int64_t je = (jb + jper < n) ? jb + jper : n;
    for (int64_t j = jb; j < je; ++j) {
        double r2[KMV64_R];
#pragma unroll
        for (int r = 0; r < KMV64_R; ++r) r2[r] = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < dl) {
                const double xjk = (double)pts[(int64_t)k * n + j];
#pragma unroll
                for (int r = 0; r < KMV64_R; ++r) {
                    const double t = xi[r][k] - xjk;
                    r2[r] = fma(t, t, r2[r]);
                }
            }
        }
        for (int k = 16; k < d; ++k) {   // dimensions beyond 16: reload row coordinates
            const double xjk = (double)pts[(int64_t)k * n + j];
#pragma unroll
            for (int r = 0; r < KMV64_R; ++r) {
                const int64_t i = rbase + (int64_t)r * KMV_THREADS;
                const int64_t ic = i < n ? i : n - 1;
                const double t = (double)pts[(int64_t)k * n + ic] - xjk;
                r2[r] = fma(t, t, r2[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < KMV64_R; ++r) {
            const double kv = kval64<KIND>(r2[r], kconst);
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[r][q] = fma(kv, u[(int64_t)q * n + j], acc[r][q]);
        }
    }
#pragma unroll
    for (int r = 0; r < KMV64_R; ++r) {
        const int64_t i = rbase + (int64_t)r * KMV_THREADS;
        if (i < n)
#pragma unroll
            for (int q = 0; q < NR; ++q) part[((int64_t)blockIdx.y * NR + q) * n + i] = acc[r][q];
    }
}

// Stage 2: y_q = scale * sum_s part[s][q] + mu u_q per column q; partials of u_q^T y_q
// in dot_part[q * gridDim.x + block].
__global__ __launch_bounds__(256) void k_kmv_finish(int64_t n, int slices, int nr,
                                                    const double* __restrict__ part,
                                                    double scale, double mu,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ y,
                                                    double* __restrict__ dot_part,
                                                    const int32_t* __restrict__ stop) {
    __shared__ double sc[4];
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (int q = 0; q < nr; ++q) {
        double dot = 0.0;
        if (i < n) {
            double s = 0.0;
            for (int z = 0; z < slices; ++z) s += part[((int64_t)z * nr + q) * n + i];
            const double ui = u[(int64_t)q * n + i];
            const double yi = fma(scale, s, mu * ui);
            y[(int64_t)q * n + i] = yi;
            dot = ui * yi;
        }
        dot = block_sum(dot, sc);
        if (threadIdx.x == 0) dot_part[(int64_t)q * gridDim.x + blockIdx.x] = dot;
    }
}

static int kmv64_slices(int64_t n) {
    const int64_t rb = (n + KMV64_ROWS - 1) / KMV64_ROWS;
    int64_t s = (2048 + rb - 1) / rb;
    const int64_t maxs = (n + 255) / 256;
    if (s > maxs) s = maxs;
    if (s < 1) s = 1;
    if (s > 256) s = 256;
    return (int)s;
}

// Float64 stage 1: ws[s][q][i] = sum over slice s of K_ij u_q[j], nr in {1, 2}.
// Returns the number of slices.
static int kmv_stage1_f64(const KernelOp& op, const double* u, int nr, double* ws,
                          const int32_t* stop, hipStream_t st) {
    const int slices = kmv64_slices(op.n);
    const int64_t jper = (op.n + slices - 1) / slices;
    dim3 grid((unsigned)((op.n + KMV64_ROWS - 1) / KMV64_ROWS), (unsigned)slices);
#define KF64(K, R) k_kmv_f64<K, R><<<grid, KMV_THREADS, 0, st>>>(op.n, op.d, op.pts, op.kconst, u, ws, jper, stop)
    if (op.kind == 1) { if (nr == 1) KF64(1, 1); else KF64(1, 2); }
    else { if (nr == 1) KF64(2, 1); else KF64(2, 2); }
#undef KF64
    return slices;
}

size_t kernel_matvec_ws_doubles(int64_t n, int d, int nr) {
    size_t w = (size_t)2 * (size_t)kmv64_slices(n) * (size_t)n;
    for (int c = 1; c <= 8; c *= 2)
        if (c == 1 || c <= nr) w = std::max(w, kernel_sym_ws_doubles(n, d, c));
    if (kernel_mma_ok(n, d))
        w = std::max(w, kernel_mma_ws_doubles(n, std::min(nr, kernel_mma_max_cols(kernel_record_len(d)))));
    w = std::max(w, kernel_sym64_ws_doubles(n, d, std::min(nr, 2)));
    return w;
}

size_t kernel_matvec_ws_doubles_for(int64_t n, int d, int nr, bool fp64) {
    if (fp64) return kernel_mma_ok(n, d) ? kernel_mma_ws_doubles(n, std::min(nr, 2))
                                         : kernel_sym64_ws_doubles(n, d, std::min(nr, 2));
    if (kernel_mma_ok(n, d))
        return kernel_mma_ws_doubles(n, std::min(nr, kernel_mma_max_cols(kernel_record_len(d))));
    size_t w = 0;
    for (int c = 1; c <= 8; c *= 2)
        if (c == 1 || c <= nr) w = std::max(w, kernel_sym_ws_doubles(n, d, c));
    return w;
}

void launch_kernel_matvec_multi(const KernelOp& op, bool fp64, const double* u, int nr, double mu,
                                double* y, double* dot_part, double* ws, const int32_t* stop,
                                hipStream_t st, bool estimate) {
    const int64_t nblk = kernel_matvec_blocks(op.n);
    for (int q0 = 0; q0 < nr;) {
        const int left = nr - q0;
        const double* uq = u + (int64_t)q0 * op.n;
        double* yq = y + (int64_t)q0 * op.n;
        double* dq = dot_part + (int64_t)q0 * nblk;
        if (fp64 && op.xd) {
            // each unordered pair once, float64 entries (Gram products on float64 MFMA
            // within the MFMA kernel's slot bound, else on the vector ALU)
            const int c = left >= 2 ? 2 : 1;
            if (kernel_mma_ok(op.n, op.d)) launch_kernel_matvec_mma64(op, uq, c, mu, yq, dq, ws, stop, st);
            else launch_kernel_matvec_sym64(op, uq, c, mu, yq, dq, ws, stop, st);
            q0 += c;
        } else if (fp64) {
            const int c = left >= 2 ? 2 : 1;
            const int slices = kmv_stage1_f64(op, uq, c, ws, stop, st);
            k_kmv_finish<<<(unsigned)nblk, 256, 0, st>>>(op.n, slices, c, ws, op.scale, mu, uq, yq, dq,
                                                         stop);
            q0 += c;
        } else if (kernel_mma_ok(op.n, op.d)) {
            // pair terms on bf16 MFMA, up to four columns at a time (two for the
            // estimate grade and the longest records): every column goes through the
            // same arithmetic whatever the block width, so a column solved alone and
            // inside a block gives bitwise the same products (this path also serves
            // the power iterations)
            const int cmax = estimate ? 2 : kernel_mma_max_cols(op.dm);
            const int c = left >= 4 && cmax >= 4 ? 4 : left >= 2 ? 2 : 1;
            launch_kernel_matvec_mma(op, uq, c, mu, yq, dq, ws, stop, st, estimate);
            q0 += c;
        } else {
            const int c = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
            launch_kernel_matvec_sym(op, uq, c, mu, yq, dq, ws, stop, st, estimate);
            q0 += c;
        }
    }
}

void launch_kernel_matvec(const KernelOp& op, bool fp64, const double* u, double mu, double* y,
                          double* dot_part, double* ws, const int32_t* stop, hipStream_t st) {
    launch_kernel_matvec_multi(op, fp64, u, 1, mu, y, dot_part, ws, stop, st);
}

// ===================================================== dense formation
template <int KIND, typename TO>
__global__ void k_kernel_to_dense(int64_t n, int d, const float* __restrict__ pts, double kconst,
                                  double scale, TO* __restrict__ out, int64_t lda) {
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, j = e / n;
        double r2 = 0.0;
        for (int k = 0; k < d; ++k) {
            const double t = (double)pts[(int64_t)k * n + i] - (double)pts[(int64_t)k * n + j];
            r2 = fma(t, t, r2);
        }
        out[i + j * lda] = from_f64<TO>(scale * kval64<KIND>(r2, kconst));
    }
}
void launch_kernel_to_dense(const KernelOp& op, void* out, int dtype, int64_t lda, hipStream_t st) {
    int64_t g = (op.n * op.n + 255) / 256;
    if (g > 65536 * 4) g = 65536 * 4;
    const int gg = (int)g;
#define KTD(K, T) k_kernel_to_dense<K, T><<<gg, 256, 0, st>>>(op.n, op.d, op.pts, op.kconst, op.scale, (T*)out, lda)
    if (op.kind == 1) {
        if (dtype == DT_F64) KTD(1, double); else if (dtype == DT_F32) KTD(1, float); else KTD(1, __hip_bfloat16);
    } else {
        if (dtype == DT_F64) KTD(2, double); else if (dtype == DT_F32) KTD(2, float); else KTD(2, __hip_bfloat16);
    }
#undef KTD
}

// ================================================ kernel-GEMM, float64 VALU
constexpr int KF_BM = 64, KF_BN = 64, KF_BK = 16;
template <int KIND>
__global__ __launch_bounds__(256) void k_kgemm_f64(int64_t n, int d, const float* __restrict__ pts,
                                                   double kconst, double scale, double mu,
                                                   const double* __restrict__ B, int64_t ldb,
                                                   int64_t m, double* __restrict__ Y,
                                                   int64_t ldy) {
    __shared__ double As[KF_BK][KF_BM + 1];
    __shared__ double Bs[KF_BK][KF_BN + 1];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * KF_BM, c0 = (int64_t)blockIdx.y * KF_BN;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += KF_BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ii = t & 63, kk = (t >> 6) + 4 * q;
            const int64_t gi = i0 + ii, gj = j0 + kk;
            double v = 0.0;
            if (gi < n && gj < n) {
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) {
                    const double dx = (double)pts[(int64_t)k * n + gi] - (double)pts[(int64_t)k * n + gj];
                    r2 = fma(dx, dx, r2);
                }
                v = kval64<KIND>(r2, kconst);
            }
            As[kk][ii] = v;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = t & 15, jj = (t >> 4) + 16 * q;
            const int64_t gj = c0 + jj, gk = j0 + kk;
            Bs[kk][jj] = (gj < m && gk < n) ? B[gk + gj * ldb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KF_BK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = As[kk][tx + 16 * u];
#pragma unroll
            for (int v = 0; v < 4; ++v) b[v] = Bs[kk][ty + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t gi = i0 + tx + 16 * u;
        if (gi >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t gc = c0 + ty + 16 * v;
            if (gc >= m) continue;
            Y[gi + gc * ldy] = fma(scale, acc[u][v], mu * B[gi + gc * ldb]);
        }
    }
}

void launch_kernel_gemm_f64(const KernelOp& op, const double* B, int64_t ldb, int64_t m, double mu,
                            double* Y, int64_t ldy, hipStream_t st) {
    dim3 grid((unsigned)((op.n + KF_BM - 1) / KF_BM), (unsigned)((m + KF_BN - 1) / KF_BN));
    if (op.kind == 1) k_kgemm_f64<1><<<grid, 256, 0, st>>>(op.n, op.d, op.pts, op.kconst, op.scale, mu, B, ldb, m, Y, ldy);
    else k_kgemm_f64<2><<<grid, 256, 0, st>>>(op.n, op.d, op.pts, op.kconst, op.scale, mu, B, ldb, m, Y, ldy);
}

}  // namespace rr
