// Dense building blocks: the float64-accumulating tiled GEMM used for the
// orthogonalisation and core products (Section 4.1-4.2, Algorithm
// prec_chol_qr), the projection kernels Q^T r and r + Q d applied every PCG
// iteration (eq. g_randrand_explicit), the stored-matrix matvec, and the CG
// vector/scalar steps (Algorithm RandRAND_PCG).  Every reduction runs in a
// fixed order, so results are bitwise reproducible run to run.
#include "common.hpp"
#include "group.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace rr {

static inline int clamp_grid(int64_t g) {
    if (g < 1) return 1;
    if (g > 1 << 20) return 1 << 20;
    return (int)g;
}

// ====================================================================== GEMM
constexpr int GBM = 64, GBN = 64, GBK = 16;

template <typename TA, typename TB, bool TRA, bool TRB>
__global__ __launch_bounds__(256) void k_gemm(int64_t M, int64_t N, int64_t K,
                                              const TA* __restrict__ A, int64_t lda,
                                              const TB* __restrict__ B, int64_t ldb,
                                              double* __restrict__ C, int64_t ldc, double alpha,
                                              double beta, int64_t kchunk,
                                              double* __restrict__ part) {
    __shared__ double As[GBK][GBM + 1];
    __shared__ double Bs[GBK][GBN + 1];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * GBM, j0 = (int64_t)blockIdx.y * GBN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;

    for (int64_t k0 = kbeg; k0 < kend; k0 += GBK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int ii, kk;
            if (!TRA) { ii = t & 63; kk = (t >> 6) + 4 * q; }
            else      { kk = t & 15; ii = (t >> 4) + 16 * q; }
            const int64_t gi = i0 + ii, gk = k0 + kk;
            double v = 0.0;
            if (gi < M && gk < kend) v = TRA ? to_f64(A[gk + gi * lda]) : to_f64(A[gi + gk * lda]);
            As[kk][ii] = v;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int kk, jj;
            if (!TRB) { kk = t & 15; jj = (t >> 4) + 16 * q; }
            else      { jj = t & 63; kk = (t >> 6) + 4 * q; }
            const int64_t gj = j0 + jj, gk = k0 + kk;
            double v = 0.0;
            if (gj < N && gk < kend) v = TRB ? to_f64(B[gj + gk * ldb]) : to_f64(B[gk + gj * ldb]);
            Bs[kk][jj] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; ++kk) {
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
    const bool split = gridDim.z > 1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t gi = i0 + tx + 16 * u;
        if (gi >= M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t gj = j0 + ty + 16 * v;
            if (gj >= N) continue;
            if (split) {
                part[(int64_t)blockIdx.z * M * N + gi + gj * M] = acc[u][v];
            } else {
                double o = alpha * acc[u][v];
                if (beta != 0.0) o += beta * C[gi + gj * ldc];
                C[gi + gj * ldc] = o;
            }
        }
    }
}

__global__ void k_gemm_reduce(int64_t M, int64_t N, int splits, const double* __restrict__ part,
                              double* __restrict__ C, int64_t ldc, double alpha, double beta) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < splits; ++z) s += part[(int64_t)z * total + e];
        const int64_t i = e % M, j = e / M;
        double o = alpha * s;
        if (beta != 0.0) o += beta * C[i + j * ldc];
        C[i + j * ldc] = o;
    }
}

template <typename TA, typename TB, bool TRA, bool TRB>
static void gemm_t(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                   int64_t ldb, double* C, int64_t ldc, double alpha, double beta, double* ws,
                   size_t ws_doubles, hipStream_t st) {
    const int64_t gm = (M + GBM - 1) / GBM, gn = (N + GBN - 1) / GBN;
    const int64_t kblocks = (K + GBK - 1) / GBK;
    int64_t splits = 1;
    const int64_t target = 1024;
    if (gm * gn < target && kblocks >= 8) {
        splits = (target + gm * gn - 1) / (gm * gn);
        if (splits > kblocks / 4) splits = kblocks / 4;
        if (splits > 64) splits = 64;
        while (splits > 1 && (size_t)(splits * M * N) > ws_doubles) --splits;
        if (splits < 1) splits = 1;
    }
    const int64_t kchunk = ((kblocks + splits - 1) / splits) * GBK;
    splits = (K + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    dim3 grid((unsigned)gm, (unsigned)gn, (unsigned)splits);
    k_gemm<TA, TB, TRA, TRB><<<grid, 256, 0, st>>>(M, N, K, (const TA*)A, lda, (const TB*)B, ldb,
                                                   C, ldc, alpha, beta, kchunk, ws);
    if (splits > 1) {
        k_gemm_reduce<<<clamp_grid((M * N + 255) / 256), 256, 0, st>>>(M, N, (int)splits, ws, C,
                                                                      ldc, alpha, beta);
    }
}

size_t gemm_ws_doubles(int64_t M, int64_t N, int64_t K) {
    (void)K;
    return (size_t)64 * (size_t)M * (size_t)N;
}

template <typename TA, typename TB>
static void gemm_tr(bool trA, bool trB, int64_t M, int64_t N, int64_t K, const void* A,
                    int64_t lda, const void* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                    double beta, double* ws, size_t wsd, hipStream_t st) {
    if (!trA && !trB) gemm_t<TA, TB, false, false>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    else if (!trA && trB) gemm_t<TA, TB, false, true>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    else if (trA && !trB) gemm_t<TA, TB, true, false>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    else gemm_t<TA, TB, true, true>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
}

// C = alpha sum_ch part[q nch M + ch M + j] + beta C: the chunk partials of a streamed
// A^T B added in chunk order.
__global__ void k_gemv_t_reduce(int64_t M, int64_t N, int nch, const double* __restrict__ part,
                                double* __restrict__ C, int64_t ldc, double alpha, double beta) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e % M, q = e / M;
        double s = 0.0;
        for (int ch = 0; ch < nch; ++ch) s += part[(q * nch + ch) * M + j];
        double o = alpha * s;
        if (beta != 0.0) o += beta * C[j + q * ldc];
        C[j + q * ldc] = o;
    }
}

void launch_gemm(int dta, bool trA, int dtb, bool trB, int64_t M, int64_t N, int64_t K,
                 const void* A, int64_t lda, const void* B, int64_t ldb, double* C, int64_t ldc,
                 double alpha, double beta, double* ws, size_t wsd, hipStream_t st) {
    if (M <= 0 || N <= 0) return;
    if (K <= 0) {  // C = beta * C
        launch_scale_mat(C, ldc, M, N, beta, st);
        return;
    }
    if (launch_gemm_mfma(dta, trA, dtb, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st))
        return;
    // A^T B with at most 8 columns of B and a long K (the Gram products of the block
    // solvers): A is streamed once per group of up to 8 columns by the projection
    // kernel's blocks (row chunks x 4 columns of A), then the partials are added.
    if (dta == DT_F64 && dtb == DT_F64 && trA && !trB && N <= 8 && K >= 1024 && ws &&
        (size_t)N * (size_t)gemv_t_chunks(K, M) * (size_t)M <= wsd) {
        const int nch = gemv_t_chunks(K, M);
        for (int64_t c0 = 0; c0 < N;) {
            const int64_t left = N - c0;
            const int nr = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
            launch_gemv_t_multi(nr, K, M, (const double*)A, lda, (const double*)B + c0 * ldb, ldb,
                                ws + c0 * nch * M, nch, nullptr, st);
            c0 += nr;
        }
        k_gemv_t_reduce<<<clamp_grid((M * N + 255) / 256), 256, 0, st>>>(M, N, nch, ws, C, ldc, alpha, beta);
        return;
    }
    if (dtb == DT_F64) {
        if (dta == DT_F64) gemm_tr<double, double>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
        else if (dta == DT_F32) gemm_tr<float, double>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
        else gemm_tr<__hip_bfloat16, double>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    } else {
        if (dta == DT_F64) gemm_tr<double, float>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
        else if (dta == DT_F32) gemm_tr<float, float>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
        else gemm_tr<__hip_bfloat16, float>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    }
}

// ================================================== small dense helpers
// out[c + i * ldo] = (double) in[i + c * ldi]: column-major in, row-major float64 out,
// through 64 x 64 LDS tiles (both sides coalesced).
template <typename TI>
__global__ __launch_bounds__(256) void k_transpose_f64(int64_t rows, int64_t cols, const TI* __restrict__ in,
                                                       int64_t ldi, double* __restrict__ out, int64_t ldo) {
    __shared__ double tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int cc = ty; cc < 64; cc += 4) {
        const int64_t i = i0 + tx, c = c0 + cc;
        if (i < rows && c < cols) tile[cc][tx] = (double)in[i + c * ldi];
    }
    __syncthreads();
#pragma unroll
    for (int ii = ty; ii < 64; ii += 4) {
        const int64_t i = i0 + ii, c = c0 + tx;
        if (i < rows && c < cols) out[c + i * ldo] = tile[tx][ii];
    }
}

void launch_transpose_f64(int dtype, int64_t rows, int64_t cols, const void* in, int64_t ldi, double* out,
                          int64_t ldo, hipStream_t st) {
    const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
    if (dtype == DT_F32)
        k_transpose_f64<float><<<grid, 256, 0, st>>>(rows, cols, (const float*)in, ldi, out, ldo);
    else
        k_transpose_f64<double><<<grid, 256, 0, st>>>(rows, cols, (const double*)in, ldi, out, ldo);
}

__global__ void k_symmetrize(double* A, int64_t l, int64_t lda) {
    const int64_t total = l * l;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % l, j = e / l;
        if (i < j) {
            const double s = 0.5 * (A[i + j * lda] + A[j + i * lda]);
            A[i + j * lda] = s;
            A[j + i * lda] = s;
        }
    }
}
void launch_symmetrize(double* A, int64_t l, int64_t lda, hipStream_t st) {
    k_symmetrize<<<clamp_grid((l * l + 255) / 256), 256, 0, st>>>(A, l, lda);
}

__global__ void k_add_diag(double* A, int64_t l, int64_t lda, double alpha, const double* adev) {
    const double a = adev ? *adev : alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < l;
         i += (int64_t)gridDim.x * blockDim.x)
        A[i + i * lda] += a;
}
void launch_add_diag(double* A, int64_t l, int64_t lda, double alpha, hipStream_t st) {
    k_add_diag<<<clamp_grid((l + 255) / 256), 256, 0, st>>>(A, l, lda, alpha, nullptr);
}
void launch_add_diag_dev(double* A, int64_t l, int64_t lda, const double* adev, hipStream_t st) {
    k_add_diag<<<clamp_grid((l + 255) / 256), 256, 0, st>>>(A, l, lda, 0.0, adev);
}

__global__ void k_two_minus(double* T, int64_t l, int64_t ldt) {
    const int64_t total = l * l;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % l, j = e / l;
        const double v = T[i + j * ldt];
        T[i + j * ldt] = (i == j ? 2.0 : 0.0) - v;
    }
}
void launch_two_minus(double* T, int64_t l, int64_t ldt, hipStream_t st) {
    k_two_minus<<<clamp_grid((l * l + 255) / 256), 256, 0, st>>>(T, l, ldt);
}

__global__ void k_zero_lower(double* A, int64_t l, int64_t lda) {
    const int64_t total = l * l;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % l, j = e / l;
        if (i > j) A[i + j * lda] = 0.0;
    }
}
void launch_zero_lower(double* A, int64_t l, int64_t lda, hipStream_t st) {
    k_zero_lower<<<clamp_grid((l * l + 255) / 256), 256, 0, st>>>(A, l, lda);
}

template <typename TS, typename TD>
__global__ void k_copy_mat(const TS* __restrict__ s, int64_t lds, TD* __restrict__ d, int64_t ldd,
                           int64_t rows, int64_t cols) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % rows, j = e / rows;
        d[i + j * ldd] = from_f64<TD>(to_f64(s[i + j * lds]));
    }
}
template <typename TS>
static void copy_from(const void* src, int64_t lds, int dtd, void* dst, int64_t ldd, int64_t rows,
                      int64_t cols, hipStream_t st) {
    const int g = clamp_grid((rows * cols + 255) / 256);
    if (dtd == DT_F64) k_copy_mat<TS, double><<<g, 256, 0, st>>>((const TS*)src, lds, (double*)dst, ldd, rows, cols);
    else if (dtd == DT_F32) k_copy_mat<TS, float><<<g, 256, 0, st>>>((const TS*)src, lds, (float*)dst, ldd, rows, cols);
    else k_copy_mat<TS, __hip_bfloat16><<<g, 256, 0, st>>>((const TS*)src, lds, (__hip_bfloat16*)dst, ldd, rows, cols);
}
void launch_copy_mat(int dts, const void* src, int64_t lds, int dtd, void* dst, int64_t ldd,
                     int64_t rows, int64_t cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    if (dts == DT_F64) copy_from<double>(src, lds, dtd, dst, ldd, rows, cols, st);
    else if (dts == DT_F32) copy_from<float>(src, lds, dtd, dst, ldd, rows, cols, st);
    else copy_from<__hip_bfloat16>(src, lds, dtd, dst, ldd, rows, cols, st);
}

__global__ void k_axpby_mat(double a, const double* __restrict__ A, int64_t lda, double b,
                            const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                            int64_t ldc, int64_t rows, int64_t cols) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % rows, j = e / rows;
        C[i + j * ldc] = a * A[i + j * lda] + b * B[i + j * ldb];
    }
}
void launch_axpby_mat(double a, const double* A, int64_t lda, double b, const double* B,
                      int64_t ldb, double* C, int64_t ldc, int64_t rows, int64_t cols,
                      hipStream_t st) {
    k_axpby_mat<<<clamp_grid((rows * cols + 255) / 256), 256, 0, st>>>(a, A, lda, b, B, ldb, C,
                                                                      ldc, rows, cols);
}

__global__ void k_scale_mat(double* A, int64_t lda, int64_t rows, int64_t cols, double s) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % rows, j = e / rows;
        A[i + j * lda] = (s == 0.0) ? 0.0 : s * A[i + j * lda];
    }
}
void launch_scale_mat(double* A, int64_t lda, int64_t rows, int64_t cols, double s, hipStream_t st) {
    k_scale_mat<<<clamp_grid((rows * cols + 255) / 256), 256, 0, st>>>(A, lda, rows, cols, s);
}

// max |M - I| over an l x l matrix: blocks take columns, threads rows; each block
// folds its maximum into *out with an integer atomicMax on the bit pattern (for
// non-negative doubles it orders like the values, so the result is exact and
// independent of the order).  *out is cleared first on the stream.
__global__ __launch_bounds__(256) void k_max_abs_minus_identity(const double* __restrict__ M, int64_t l,
                                                                int64_t ldm, unsigned long long* out) {
    __shared__ double sh[256 / WAVE];
    double m = 0.0;
    for (int64_t j = blockIdx.x; j < l; j += gridDim.x)
        for (int64_t i = threadIdx.x; i < l; i += blockDim.x) {
            const double v = fabs(M[i + j * ldm] - (i == j ? 1.0 : 0.0));
            m = v > m ? v : m;
        }
    for (int o = WAVE / 2; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sh[0];
        for (int w = 1; w < 256 / WAVE; ++w) b = fmax(b, sh[w]);
        atomicMax(out, (unsigned long long)__double_as_longlong(b));
    }
}
void launch_max_abs_minus_identity(const double* M, int64_t l, int64_t ldm, double* out,
                                   hipStream_t st) {
    (void)hipMemsetAsync(out, 0, sizeof(double), st);
    const int g = (int)std::min<int64_t>(std::max<int64_t>(l, 1), 1024);
    k_max_abs_minus_identity<<<g, 256, 0, st>>>(M, l, ldm, (unsigned long long*)out);
}

// ============================================ stored dense matvec (K5)
// y_j = sum_i A[i, j] u_i (A symmetric, so this is (A u)_j) + mu u_j.  A block of
// 256 threads owns DM_COLS consecutive columns: every column is read as one
// contiguous, coalesced stream, the u values a thread loads are reused across
// the block's columns, and the products are accumulated in float64.
constexpr int DM_THREADS = 256;

template <typename TA, int DM_COLS>
__global__ __launch_bounds__(DM_THREADS) void k_dense_matvec(int64_t n, const TA* __restrict__ A,
                                                             int64_t lda,
                                                             const double* __restrict__ u,
                                                             double mu, double* __restrict__ y,
                                                             double* __restrict__ dot_part,
                                                             const int32_t* __restrict__ stop) {
    __shared__ double red[DM_COLS][DM_THREADS / WAVE];
    if (stop && *stop) return;
    const int64_t j0 = (int64_t)blockIdx.x * DM_COLS;
    double acc[DM_COLS];
#pragma unroll
    for (int c = 0; c < DM_COLS; ++c) acc[c] = 0.0;
    constexpr int VW = 16 / sizeof(TA);   // elements per 16-byte load
    const bool vec_ok = (lda % VW) == 0 && (((uintptr_t)A) & 15) == 0;
    int64_t i_start = 0;
    if (vec_ok) {
        const int64_t nv = n / VW;
        for (int64_t v = threadIdx.x; v < nv; v += DM_THREADS) {
            double uu[VW];
#pragma unroll
            for (int w = 0; w < VW; ++w) uu[w] = u[v * VW + w];
#pragma unroll
            for (int c = 0; c < DM_COLS; ++c) {
                const int64_t j = j0 + c;
                if (j < n) {
                    // large n: A streams through once, so non-temporal loads keep u in the
                    // caches (a small matrix stays cache-resident across iterations instead)
                    const TA* col = A + j * lda + v * VW;
                    if constexpr (sizeof(TA) == 4) {
                        typedef float f4v __attribute__((ext_vector_type(4)));
                        const f4v a = DM_COLS >= 16 ? __builtin_nontemporal_load(reinterpret_cast<const f4v*>(col))
                                                    : *reinterpret_cast<const f4v*>(col);
                        acc[c] = fma((double)a[0], uu[0], acc[c]);
                        acc[c] = fma((double)a[1], uu[1], acc[c]);
                        acc[c] = fma((double)a[2], uu[2], acc[c]);
                        acc[c] = fma((double)a[3], uu[3], acc[c]);
                    } else {
                        typedef double d2v __attribute__((ext_vector_type(2)));
                        const d2v a = DM_COLS >= 16 ? __builtin_nontemporal_load(reinterpret_cast<const d2v*>(col))
                                                    : *reinterpret_cast<const d2v*>(col);
                        acc[c] = fma(a[0], uu[0], acc[c]);
                        acc[c] = fma(a[1], uu[1], acc[c]);
                    }
                }
            }
        }
        i_start = nv * VW;
    }
    for (int64_t i = i_start + threadIdx.x; i < n; i += DM_THREADS) {
        const double ui = u[i];
#pragma unroll
        for (int c = 0; c < DM_COLS; ++c) {
            const int64_t j = j0 + c;
            if (j < n) acc[c] = fma(to_f64(A[i + j * lda]), ui, acc[c]);
        }
    }
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int c = 0; c < DM_COLS; ++c) {
        const double s = wave_sum(acc[c]);
        if (lane == 0) red[c][w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double dot = 0.0;
        for (int c = 0; c < DM_COLS; ++c) {
            const int64_t j = j0 + c;
            if (j >= n) break;
            double s = 0.0;
            for (int q = 0; q < DM_THREADS / WAVE; ++q) s += red[c][q];
            const double yj = s + mu * u[j];
            y[j] = yj;
            dot = fma(u[j], yj, dot);
        }
        dot_part[blockIdx.x] = dot;
    }
}

// Columns per block: 16 for large n (each u chunk read from cache serves 16 columns);
// 2 below 8,192, so a small matrix still spreads over every compute unit.  A column's
// sum is formed the same way either way (each thread's strided terms, then the block
// reduction in a fixed order).
static int dense_matvec_cols(int64_t n) { return n <= 8192 ? 2 : 16; }
int dense_matvec_blocks(int64_t n) {
    const int c = dense_matvec_cols(n);
    return (int)((n + c - 1) / c);
}

void launch_dense_matvec(int dta, int64_t n, const void* A, int64_t lda, const double* u,
                         double mu, double* y, double* dot_part, const int32_t* stop,
                         hipStream_t st) {
    const int g = dense_matvec_blocks(n);
    ProfScope prof(dta == DT_F32 ? PROF_DENSE_MATVEC : PROF_DENSE_MATVEC64, st);
#define KDM(T, C) k_dense_matvec<T, C><<<g, DM_THREADS, 0, st>>>(n, (const T*)A, lda, u, mu, y, dot_part, stop)
    if (dense_matvec_cols(n) == 2) {
        if (dta == DT_F32) KDM(float, 2); else KDM(double, 2);
    } else {
        if (dta == DT_F32) KDM(float, 16); else KDM(double, 16);
    }
#undef KDM
}

// ============================================== projections
// C[:, q] = Q^T R[:, q] and Z[:, q] = rcoef_q R[:, q] + Q D[:, q] for NR = 1 or 2
// vectors at once, so Q (n x k, the HBM-bound operand) is read once for both.

// c_part[q * nchunks * k + ch * k + j] = sum over rows of chunk ch of Q[i, j] R[i, q].
constexpr int GT_COLS = 4;
constexpr int GT_THREADS = 256;

// Block (bx, ch): columns GT_COLS bx .. of Q over row chunk ch (shared with the
// grouped serving kernel).
template <int NR>
RR_DEV void gemv_t_block(int bx, int ch, int64_t n, int64_t k, const double* __restrict__ Q, int64_t ldq,
                         const double* __restrict__ R, int64_t ldr, double* __restrict__ c_part, int nchunks,
                         int64_t rows_per_chunk) {
    __shared__ double red[GT_COLS * NR][GT_THREADS / WAVE];
    const int64_t j0 = (int64_t)bx * GT_COLS;
    const int64_t ib = ch * rows_per_chunk;
    const int64_t ie = (ib + rows_per_chunk < n) ? ib + rows_per_chunk : n;
    double acc[GT_COLS][NR];
#pragma unroll
    for (int c = 0; c < GT_COLS; ++c)
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[c][q] = 0.0;
    // two rows per thread per pass: eight independent loads of Q in flight
    const int ncol = (int)((k - j0) < GT_COLS ? (k - j0) : GT_COLS);
    int64_t i = ib + threadIdx.x;
    for (; i + GT_THREADS < ie; i += 2 * GT_THREADS) {
        double ri[2][NR], qv[2][GT_COLS];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int q = 0; q < NR; ++q) ri[h][q] = R[i + h * GT_THREADS + q * ldr];
#pragma unroll
            for (int c = 0; c < GT_COLS; ++c)
                qv[h][c] = c < ncol ? Q[i + h * GT_THREADS + (j0 + c) * ldq] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < GT_COLS; ++c)
#pragma unroll
                for (int q = 0; q < NR; ++q) acc[c][q] = fma(qv[h][c], ri[h][q], acc[c][q]);
    }
    for (; i < ie; i += GT_THREADS) {
        double ri[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) ri[q] = R[i + q * ldr];
#pragma unroll
        for (int c = 0; c < GT_COLS; ++c)
            if (c < ncol) {
                const double qij = Q[i + (j0 + c) * ldq];
#pragma unroll
                for (int q = 0; q < NR; ++q) acc[c][q] = fma(qij, ri[q], acc[c][q]);
            }
    }
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int c = 0; c < GT_COLS; ++c)
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const double s = wave_sum(acc[c][q]);
            if (lane == 0) red[c * NR + q][w] = s;
        }
    __syncthreads();
    if (threadIdx.x < GT_COLS * NR) {
        const int c = threadIdx.x / NR, q = threadIdx.x % NR;
        const int64_t j = j0 + c;
        if (j < k) {
            double s = 0.0;
            for (int w2 = 0; w2 < GT_THREADS / WAVE; ++w2) s += red[threadIdx.x][w2];
            c_part[(int64_t)q * nchunks * k + (int64_t)ch * k + j] = s;
        }
    }
}
template <int NR>
__global__ __launch_bounds__(GT_THREADS) void k_gemv_t(int64_t n, int64_t k,
                                                       const double* __restrict__ Q, int64_t ldq,
                                                       const double* __restrict__ R, int64_t ldr,
                                                       double* __restrict__ c_part, int nchunks,
                                                       int64_t rows_per_chunk,
                                                       const int32_t* __restrict__ stop) {
    if (stop && *stop) return;
    gemv_t_block<NR>(blockIdx.x, blockIdx.y, n, k, Q, ldq, R, ldr, c_part, nchunks, rows_per_chunk);
}

static int64_t gemv_t_rows_per_chunk(int64_t n, int64_t k) {
    const int64_t colblocks = (k + GT_COLS - 1) / GT_COLS;
    int64_t chunks = (2048 + colblocks - 1) / colblocks;
    const int64_t max_chunks = (n + 1023) / 1024;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    if (chunks > 64) chunks = 64;
    return (n + chunks - 1) / chunks;
}

int64_t gemv_t_rows_per_chunk_of(int64_t n, int64_t k) { return gemv_t_rows_per_chunk(n, k); }

int gemv_t_chunks(int64_t n, int64_t k) {
    const int64_t rpc = gemv_t_rows_per_chunk(n, k);
    return (int)((n + rpc - 1) / rpc);
}

void launch_gemv_t_multi(int nr, int64_t n, int64_t k, const double* Q, int64_t ldq, const double* R,
                         int64_t ldr, double* c_part, int nchunks, const int32_t* stop, hipStream_t st) {
    const int64_t rpc = gemv_t_rows_per_chunk(n, k);
    dim3 grid((unsigned)((k + GT_COLS - 1) / GT_COLS), (unsigned)nchunks);
    switch (nr) {
        case 8: k_gemv_t<8><<<grid, GT_THREADS, 0, st>>>(n, k, Q, ldq, R, ldr, c_part, nchunks, rpc, stop); break;
        case 4: k_gemv_t<4><<<grid, GT_THREADS, 0, st>>>(n, k, Q, ldq, R, ldr, c_part, nchunks, rpc, stop); break;
        case 2: k_gemv_t<2><<<grid, GT_THREADS, 0, st>>>(n, k, Q, ldq, R, ldr, c_part, nchunks, rpc, stop); break;
        default: k_gemv_t<1><<<grid, GT_THREADS, 0, st>>>(n, k, Q, ldq, R, ldr, c_part, nchunks, rpc, stop); break;
    }
}
void launch_gemv_t(int64_t n, int64_t k, const double* Q, int64_t ldq, const double* r,
                   double* c_part, int nchunks, const int32_t* stop, hipStream_t st) {
    launch_gemv_t_multi(1, n, k, Q, ldq, r, n, c_part, nchunks, stop, st);
}

// d_i = sum_j Kc[j, i] c_j with c_j = sum_ch c_part[ch*k + j] (Kc symmetric).
// blockIdx.y = column q of a pair (core K0 or K1, its own c_part and d slices).
// Each thread finishes the c_j of its own j (partials added in chunk order) and
// uses them at once, so the block needs no staging barrier.
constexpr int CA_ROWS = 4;
// blockIdx.y = 2 (launch_core_apply_triple): core K2 on column 1's c, into d[2k:3k);
// c_out, when given, receives column 1's c.
// Block (bx, q): rows CA_ROWS bx .. of d for column q (shared with the grouped
// serving kernel).
RR_DEV void core_apply_block(int bx, int q, int64_t k, const double* __restrict__ K0,
                             const double* __restrict__ K1, int64_t ldk, const double* __restrict__ c_part,
                             int nchunks, double* __restrict__ d, const double* __restrict__ K2,
                             double* __restrict__ c_out, bool shared_core) {
    __shared__ double red[CA_ROWS][256 / WAVE];
    // shared_core: column q of c_part with core K0 (any number of columns);
    // otherwise the pair / triple layout above
    const double* __restrict__ Kc = shared_core ? K0 : q == 0 ? K0 : q == 1 ? K1 : K2;
    const double* __restrict__ cp = c_part + (int64_t)(shared_core ? q : (q ? 1 : 0)) * nchunks * k;
    const bool write_c = c_out && q == 1 && bx == 0;
    const int64_t i0 = (int64_t)bx * CA_ROWS;
    double acc[CA_ROWS];
#pragma unroll
    for (int r = 0; r < CA_ROWS; ++r) acc[r] = 0.0;
    for (int64_t j = threadIdx.x; j < k; j += blockDim.x) {
        double kv[CA_ROWS];
#pragma unroll
        for (int r = 0; r < CA_ROWS; ++r) kv[r] = (i0 + r < k) ? Kc[j + (i0 + r) * ldk] : 0.0;
        double cj = 0.0;
        int ch = 0;
        for (; ch + 4 <= nchunks; ch += 4) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = cp[(int64_t)(ch + u) * k + j];
#pragma unroll
            for (int u = 0; u < 4; ++u) cj += v[u];
        }
        for (; ch < nchunks; ++ch) cj += cp[(int64_t)ch * k + j];
        if (write_c) c_out[j] = cj;
#pragma unroll
        for (int r = 0; r < CA_ROWS; ++r) acc[r] = fma(kv[r], cj, acc[r]);
    }
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int r = 0; r < CA_ROWS; ++r) {
        const double s = wave_sum(acc[r]);
        if (lane == 0) red[r][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < CA_ROWS && i0 + threadIdx.x < k) {
        double s = 0.0;
        for (int w2 = 0; w2 < 256 / WAVE; ++w2) s += red[threadIdx.x][w2];
        d[(int64_t)q * k + i0 + threadIdx.x] = s;
    }
}
__global__ __launch_bounds__(256) void k_core_apply(int64_t k, const double* __restrict__ K0,
                                                    const double* __restrict__ K1, int64_t ldk,
                                                    const double* __restrict__ c_part, int nchunks,
                                                    double* __restrict__ d,
                                                    const int32_t* __restrict__ stop,
                                                    const double* __restrict__ K2 = nullptr,
                                                    double* __restrict__ c_out = nullptr,
                                                    bool shared_core = false) {
    if (stop && *stop) return;
    core_apply_block(blockIdx.x, blockIdx.y, k, K0, K1, ldk, c_part, nchunks, d, K2, c_out, shared_core);
}

void launch_core_apply(int64_t k, const double* Kc, int64_t ldk, const double* c_part,
                       int nchunks, double* d, const int32_t* stop, hipStream_t st) {
    const int g = (int)((k + CA_ROWS - 1) / CA_ROWS);
    k_core_apply<<<dim3(g, 1), 256, 0, st>>>(k, Kc, Kc, ldk, c_part, nchunks, d, stop);
}
void launch_core_apply_pair(int64_t k, const double* K0, const double* K1, int64_t ldk,
                            const double* c_part, int nchunks, double* d, const int32_t* stop,
                            hipStream_t st) {
    const int g = (int)((k + CA_ROWS - 1) / CA_ROWS);
    k_core_apply<<<dim3(g, 2), 256, 0, st>>>(k, K0, K1, ldk, c_part, nchunks, d, stop);
}
void launch_core_apply_cols(int64_t k, const double* Kc, int64_t ldk, const double* c_part, int nchunks,
                            int ncols, double* d, hipStream_t st) {
    const int g = (int)((k + CA_ROWS - 1) / CA_ROWS);
    k_core_apply<<<dim3(g, ncols), 256, 0, st>>>(k, Kc, Kc, ldk, c_part, nchunks, d, nullptr, Kc, nullptr,
                                                 true);
}
void launch_core_apply_triple(int64_t k, const double* K0, const double* K1, const double* K2, int64_t ldk,
                              const double* c_part, int nchunks, double* d, double* c1_out, hipStream_t st) {
    const int g = (int)((k + CA_ROWS - 1) / CA_ROWS);
    k_core_apply<<<dim3(g, 3), 256, 0, st>>>(k, K0, K1, ldk, c_part, nchunks, d, nullptr, K2, c1_out);
}

// Z[i, q] = rcoef_q R[i, q] + sum_j Q[i, j] D[j, q]; partial sums of R[i, q] Z[i, q]
// per block in rz_part[q * gridDim.x + block].  Block: 64 rows, its four waves
// split the k columns (lane = row, loads of Q coalesced along the column) and add
// their partial row sums in a fixed order.
constexpr int QD_ROWS = 64;
constexpr int QD_THREADS = 256;
// Block bx of the nblk row blocks; d_sh: LDS for NR * k doubles (shared with the
// grouped serving kernel).
template <int NR>
RR_DEV void qd_block(int bx, int nblk, int64_t n, int64_t k, const double* __restrict__ Q, int64_t ldq,
                     const double* __restrict__ D, const double* __restrict__ R, int64_t ldr, double rc0,
                     double rc1, double* __restrict__ Z, double* __restrict__ rz_part, double* d_sh) {
    __shared__ double part[QD_THREADS / WAVE][NR][QD_ROWS];
    for (int64_t e = threadIdx.x; e < (int64_t)NR * k; e += QD_THREADS) d_sh[e] = D[e];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int64_t i = (int64_t)bx * QD_ROWS + lane;
    const int64_t per = (k + 3) / 4;
    const int64_t jb = w * per, je = (jb + per < k) ? jb + per : k;
    double acc[NR][2];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q][0] = acc[q][1] = 0.0;
    if (i < n) {
        const double* qi = Q + i;
        int64_t j = jb;
        for (; j + 8 <= je; j += 8) {
            double qv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) qv[u] = qi[(j + u) * ldq];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q) acc[q][u & 1] = fma(qv[u], d_sh[q * k + j + u], acc[q][u & 1]);
        }
        for (; j < je; ++j) {
            const double qv = qi[j * ldq];
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[q][0] = fma(qv, d_sh[q * k + j], acc[q][0]);
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) part[w][q][lane] = acc[q][0] + acc[q][1];
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            double rz = 0.0;
            if (i < n) {
                const double s = (part[0][q][lane] + part[1][q][lane]) + (part[2][q][lane] + part[3][q][lane]);
                const double ri = R[i + q * ldr];
                const double zi = fma(q == 0 ? rc0 : rc1, ri, s);
                Z[i + q * ldr] = zi;
                rz = ri * zi;
            }
            rz = wave_sum(rz);
            if (lane == 0) rz_part[(int64_t)q * nblk + bx] = rz;
        }
    }
}
template <int NR>
__global__ __launch_bounds__(QD_THREADS) void k_qd(int64_t n, int64_t k,
                                                   const double* __restrict__ Q, int64_t ldq,
                                                   const double* __restrict__ D,
                                                   const double* __restrict__ R, int64_t ldr,
                                                   double rc0, double rc1,
                                                   double* __restrict__ Z,
                                                   double* __restrict__ rz_part,
                                                   const int32_t* __restrict__ stop) {
    extern __shared__ double d_sh[];   // NR * k
    if (stop && *stop) return;
    qd_block<NR>(blockIdx.x, gridDim.x, n, k, Q, ldq, D, R, ldr, rc0, rc1, Z, rz_part, d_sh);
}

int qd_blocks(int64_t n) { return (int)((n + QD_ROWS - 1) / QD_ROWS); }

void launch_qd_multi(int nr, int64_t n, int64_t k, const double* Q, int64_t ldq, const double* D,
                     const double* R, int64_t ldr, double rc0, double rc1, double* Z, double* rz_part,
                     const int32_t* stop, hipStream_t st) {
    const size_t shm = (size_t)std::max<int64_t>(nr * k, 1) * sizeof(double);
    switch (nr) {
        case 8: k_qd<8><<<qd_blocks(n), QD_THREADS, shm, st>>>(n, k, Q, ldq, D, R, ldr, rc0, rc1, Z, rz_part, stop); break;
        case 4: k_qd<4><<<qd_blocks(n), QD_THREADS, shm, st>>>(n, k, Q, ldq, D, R, ldr, rc0, rc1, Z, rz_part, stop); break;
        case 2: k_qd<2><<<qd_blocks(n), QD_THREADS, shm, st>>>(n, k, Q, ldq, D, R, ldr, rc0, rc1, Z, rz_part, stop); break;
        default: k_qd<1><<<qd_blocks(n), QD_THREADS, shm, st>>>(n, k, Q, ldq, D, R, ldr, rc0, rc1, Z, rz_part, stop); break;
    }
}
void launch_qd(int64_t n, int64_t k, const double* Q, int64_t ldq, const double* d,
               const double* r, double rcoef, double* z, double* rz_part, const int32_t* stop,
               hipStream_t st) {
    launch_qd_multi(1, n, k, Q, ldq, d, r, n, rcoef, 0.0, z, rz_part, stop, st);
}

// ==================================================== CG vector steps (K10)
constexpr int VB = 256;
int vec_blocks(int64_t n) {
    int64_t g = (n + VB * 4 - 1) / (VB * 4);
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return (int)g;
}

__global__ __launch_bounds__(VB) void k_xr_update(int64_t n, double* __restrict__ x,
                                                  double* __restrict__ r,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ w, CgState* s,
                                                  double* __restrict__ rr_part) {
    __shared__ double sc[VB / WAVE];
    if (s->stop) return;
    const double a = s->alpha;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        x[i] = fma(a, p[i], x[i]);
        const double ri = fma(-a, w[i], r[i]);
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = acc;
}
void launch_xr_update(int64_t n, double* x, double* r, const double* p, const double* w,
                      CgState* s, double* rr_part, hipStream_t st) {
    k_xr_update<<<vec_blocks(n), VB, 0, st>>>(n, x, r, p, w, s, rr_part);
}

__global__ __launch_bounds__(VB) void k_p_update(int64_t n, const double* __restrict__ z,
                                                 double* __restrict__ p, const CgState* s) {
    if (s->stop) return;
    const double b = s->beta;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        p[i] = fma(b, p[i], z[i]);
}
void launch_p_update(int64_t n, const double* z, double* p, const CgState* s, hipStream_t st) {
    k_p_update<<<vec_blocks(n), VB, 0, st>>>(n, z, p, s);
}

__global__ __launch_bounds__(VB) void k_residual(int64_t n, const double* __restrict__ b,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ r,
                                                 double* __restrict__ rr_part) {
    __shared__ double sc[VB / WAVE];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        const double ri = b[i] - w[i];
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = acc;
}
void launch_residual(int64_t n, const double* b, const double* w, double* r, double* rr_part,
                     hipStream_t st) {
    k_residual<<<vec_blocks(n), VB, 0, st>>>(n, b, w, r, rr_part);
}

__global__ void k_copy_vec(int64_t n, const double* __restrict__ s, double* __restrict__ d) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        d[i] = s[i];
}
void launch_copy_vec(int64_t n, const double* src, double* dst, hipStream_t st) {
    k_copy_vec<<<vec_blocks(n), VB, 0, st>>>(n, src, dst);
}

__global__ __launch_bounds__(VB) void k_dot_part(int64_t n, const double* __restrict__ a,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ part) {
    __shared__ double sc[VB / WAVE];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        acc = fma(a[i], b[i], acc);
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
void launch_dot_part(int64_t n, const double* a, const double* b, double* part, hipStream_t st) {
    k_dot_part<<<vec_blocks(n), VB, 0, st>>>(n, a, b, part);
}

// ----------------------------------------------------- scalar steps
__global__ void k_scal_alpha(const double* __restrict__ part, int count, CgState* s) {
    __shared__ double sc[16];
    if (s->stop) return;
    const double pw = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) {
        s->pw = pw;
        if (!(pw > 0.0) || !isfinite(pw)) {
            s->stop = STOP_BREAKDOWN;
        } else {
            s->alpha = s->rho / pw;
        }
    }
}
void launch_scal_alpha(const double* part, int count, CgState* s, hipStream_t st) {
    k_scal_alpha<<<1, 1024, 0, st>>>(part, count, s);
}

__global__ void k_scal_rr(const double* __restrict__ part, int count, CgState* s) {
    __shared__ double sc[16];
    if (s->stop) return;
    const double rr = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) {
        s->rr = rr;
        const int it = s->iters + 1;
        s->iters = it;
        if (s->hist && it < s->hist_cap) s->hist[it] = rr;
        if (!isfinite(rr)) s->stop = STOP_BREAKDOWN;
        else if (rr <= s->target2) s->stop = STOP_TARGET;
        else if (it >= s->maxit) s->stop = STOP_MAXIT;
    }
}
void launch_scal_rr(const double* part, int count, CgState* s, hipStream_t st) {
    k_scal_rr<<<1, 1024, 0, st>>>(part, count, s);
}

__global__ void k_scal_beta(const double* __restrict__ part, int count, CgState* s) {
    __shared__ double sc[16];
    if (s->stop) return;
    const double rz = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) {
        if (!(rz > 0.0) || !isfinite(rz)) {
            s->stop = STOP_BREAKDOWN;
        } else {
            s->beta = rz / s->rho;
            s->rho = rz;
        }
    }
}
void launch_scal_beta(const double* part, int count, CgState* s, hipStream_t st) {
    k_scal_beta<<<1, 1024, 0, st>>>(part, count, s);
}

__global__ void k_scal_set(const double* __restrict__ part, int count, double* out) {
    __shared__ double sc[16];
    const double v = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) *out = v;
}
void launch_scal_set(const double* part, int count, double* out, hipStream_t st) {
    k_scal_set<<<1, 1024, 0, st>>>(part, count, out);
}

__global__ void k_state_init(CgState* s, const double* __restrict__ rz_part, int rz_count,
                             double target2, int32_t maxit, int32_t iters, double* hist,
                             int32_t hist_cap) {
    __shared__ double sc[16];
    const double rz = block_sum_array(rz_part, rz_count, sc);
    if (threadIdx.x == 0) {
        s->alpha = 0.0;
        s->beta = 0.0;
        s->rho = rz;
        s->pw = 0.0;
        s->target2 = target2;
        s->iters = iters;
        s->maxit = maxit;
        s->hist = hist;
        s->hist_cap = hist_cap;
        s->stop = (!(rz > 0.0) || !isfinite(rz)) ? STOP_BREAKDOWN : STOP_NONE;
    }
}
void launch_state_init(CgState* s, const double* rz_part, int rz_count, double target2,
                       int32_t maxit, int32_t iters, double* hist, int32_t hist_cap,
                       hipStream_t st) {
    k_state_init<<<1, 1024, 0, st>>>(s, rz_part, rz_count, target2, maxit, iters, hist, hist_cap);
}

__global__ void k_nonfinite(int64_t n, const double* __restrict__ v, int32_t* flag, int32_t* nonzero) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = v[i];
        if (!isfinite(x)) *flag = 1;
        if (nonzero && x != 0.0) *nonzero = 1;
    }
}
void launch_nonfinite(int64_t n, const double* v, int32_t* flag, hipStream_t st, int32_t* nonzero) {
    k_nonfinite<<<vec_blocks(n), 256, 0, st>>>(n, v, flag, nonzero);
}

}  // namespace rr

namespace rr {
// v = src / ||src|| with ||src||^2 = sum(part) (fixed-order sum in every block);
// block 0 stores ||src|| in lam_out.
__global__ __launch_bounds__(256) void k_normalize(int64_t n, double* __restrict__ v,
                                                   const double* __restrict__ src,
                                                   const double* __restrict__ part, int count,
                                                   double* lam_out) {
    __shared__ double sc[4];
    const double s = block_sum_array(part, count, sc);
    const double nrm = sqrt(s > 0.0 ? s : 0.0);   // a y^T (I-Pi)^2 y may round below zero
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *lam_out = nrm;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        v[i] = src[i] * inv;
}
void launch_normalize(int64_t n, double* v, const double* src, const double* part, int count,
                      double* lam_out, hipStream_t st) {
    k_normalize<<<vec_blocks(n), 256, 0, st>>>(n, v, src, part, count, lam_out);
}

// Two normalisations in one launch (blockIdx.y = column): column 0 as k_normalize;
// column 1 with ||src1||^2 = a^T b over k entries, summed in every block in a fixed order.
__global__ __launch_bounds__(256) void k_normalize_pair(int64_t n, double* __restrict__ v0,
                                                        const double* __restrict__ src0,
                                                        const double* __restrict__ part0, int count0,
                                                        double* lam0, double* __restrict__ v1,
                                                        const double* __restrict__ src1,
                                                        const double* __restrict__ a,
                                                        const double* __restrict__ b, int64_t k,
                                                        double* lam1) {
    __shared__ double sc[4];
    const bool second = blockIdx.y == 1;
    double s;
    if (!second) {
        s = block_sum_array(part0, count0, sc);
    } else {
        double t = 0.0;
        for (int64_t j = threadIdx.x; j < k; j += 256) t = fma(a[j], b[j], t);
        s = block_sum(t, sc);
    }
    const double nrm = sqrt(s > 0.0 ? s : 0.0);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    double* v = second ? v1 : v0;
    const double* src = second ? src1 : src0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *(second ? lam1 : lam0) = nrm;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        v[i] = src[i] * inv;
}
void launch_normalize_pair(int64_t n, double* v0, const double* src0, const double* part0, int count0,
                           double* lam0, double* v1, const double* src1, const double* a, const double* b,
                           int64_t k, double* lam1, hipStream_t st) {
    k_normalize_pair<<<dim3((unsigned)vec_blocks(n), 2), 256, 0, st>>>(n, v0, src0, part0, count0, lam0, v1,
                                                                        src1, a, b, k, lam1);
}

// ------------------------------------------------------------------ grouped
// The projection of many column groups (of many requests) in one persistent launch
// per kernel and width: a group's items are the blocks k_gemv_t, k_core_apply and
// k_qd would run for it.  Groups whose columns have all stopped are skipped.
RR_DEV bool group_proj_runs(const GProj& g) {
    const BState* st = gu(g.st);
    const int32_t nr = gu(g.nr);
    for (int32_t q = 0; q < nr; ++q)
        if (gu(st[q].run)) return true;
    return false;
}

template <int NR>
__global__ __launch_bounds__(GT_THREADS) void k_group_gemv(const GTable* __restrict__ tab, int list,
                                                           const GProj* __restrict__ units, int32_t* ctr) {
    __shared__ int32_t wsh;
    const int32_t off = gu(tab->list[list].off), cnt = gu(tab->list[list].count);
    const int32_t total = gu(tab->list[list].total);
    GroupCursor cur(ctr, &wsh);
    while (true) {
        const int32_t w = cur.next();
        if (w >= total) return;
        const int32_t ui = group_find(units, off, off + cnt, w, [](const GProj& g) { return g.w_gemv; });
        const GProj& g = units[ui];
        if (!group_proj_runs(g)) continue;
        const int32_t cblk = gu(g.cblk), loc = w - gu(g.w_gemv);
        const int64_t n = gu(g.n);
        gemv_t_block<NR>(loc % cblk, loc / cblk, n, gu(g.k), gu(g.Q), n, gu(g.R), n, gu(g.cpart), gu(g.nch),
                         gu(g.rpc));
    }
}

__global__ __launch_bounds__(256) void k_group_core(const GTable* __restrict__ tab,
                                                    const GProj* __restrict__ units, int32_t* ctr) {
    __shared__ int32_t wsh;
    const int32_t off = gu(tab->list[GL_CORE].off), cnt = gu(tab->list[GL_CORE].count);
    const int32_t total = gu(tab->list[GL_CORE].total);
    GroupCursor cur(ctr, &wsh);
    while (true) {
        const int32_t w = cur.next();
        if (w >= total) return;
        const int32_t ui = group_find(units, off, off + cnt, w, [](const GProj& g) { return g.w_core; });
        const GProj& g = units[ui];
        if (!group_proj_runs(g)) continue;
        const int64_t k = gu(g.k);
        const int32_t rb = (int32_t)((k + CA_ROWS - 1) / CA_ROWS), loc = w - gu(g.w_core);
        const double* Kc = gu(g.Kc);
        core_apply_block(loc % rb, loc / rb, k, Kc, Kc, k, gu(g.cpart), gu(g.nch), gu(g.D), Kc, nullptr, true);
    }
}

template <int NR>
__global__ __launch_bounds__(QD_THREADS) void k_group_qd(const GTable* __restrict__ tab, int list,
                                                         const GProj* __restrict__ units, int32_t* ctr) {
    extern __shared__ double d_sh[];   // NR * group_qd_kmax(NR)
    __shared__ int32_t wsh;
    const int32_t off = gu(tab->list[list].off), cnt = gu(tab->list[list].count);
    const int32_t total = gu(tab->list[list].total);
    GroupCursor cur(ctr, &wsh);
    while (true) {
        const int32_t w = cur.next();
        if (w >= total) return;
        const int32_t ui = group_find(units, off, off + cnt, w, [](const GProj& g) { return g.w_qd; });
        const GProj& g = units[ui];
        if (!group_proj_runs(g)) continue;
        const int64_t n = gu(g.n);
        qd_block<NR>(w - gu(g.w_qd), gu(g.nbq), n, gu(g.k), gu(g.Q), n, gu(g.D), gu(g.R), n, 1.0, 1.0, gu(g.Z),
                     gu(g.rz), d_sh);
    }
}

void launch_group_proj(int list, int blocks, const GTable* tab, const GProj* projs, int32_t* ctr, hipStream_t st) {
    if (list == GL_CORE) {
        k_group_core<<<blocks, 256, 0, st>>>(tab, projs, ctr);
    } else if (list >= GL_GEMV && list < GL_GEMV + 4) {
        switch (list - GL_GEMV) {
            case 3: k_group_gemv<8><<<blocks, GT_THREADS, 0, st>>>(tab, list, projs, ctr); break;
            case 2: k_group_gemv<4><<<blocks, GT_THREADS, 0, st>>>(tab, list, projs, ctr); break;
            case 1: k_group_gemv<2><<<blocks, GT_THREADS, 0, st>>>(tab, list, projs, ctr); break;
            default: k_group_gemv<1><<<blocks, GT_THREADS, 0, st>>>(tab, list, projs, ctr); break;
        }
    } else {
#define KGQ(R) k_group_qd<R><<<blocks, QD_THREADS, (size_t)R * group_qd_kmax(R) * sizeof(double), st>>>(tab, list, projs, ctr)
        switch (list - GL_QD) {
            case 3: KGQ(8); break;
            case 2: KGQ(4); break;
            case 1: KGQ(2); break;
            default: KGQ(1); break;
        }
#undef KGQ
    }
}
}  // namespace rr
