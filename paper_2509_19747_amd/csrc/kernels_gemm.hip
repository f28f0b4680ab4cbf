// Dense float64 GEMM on v_mfma_f64_16x16x4_f64: C = alpha op(A) op(B) + beta C with
// float64 or float32 inputs (widened exactly) and float64 accumulation.  These are
// the block products of the build (Theta Y, Y R^{-1}, W^T W, Omega^T Y, Q^T Q, the
// per-shift projections of the joint basis, the blocked Householder updates).
//
// Block: 256 threads = 4 waves in a 2 x 2 grid of 32 x 32 wave tiles (2 x 2 MFMA
// tiles each, 16 float64 accumulators per lane); block tile 64 x 64; k step 16.
// The small tile keeps registers low so several blocks share a compute unit: the
// float64 MFMA pipe needs several resident waves per SIMD to stay busy.
// The next k step's tiles are loaded into registers while the current one is
// multiplied from LDS.  Skinny products (few output tiles, long K) split K over
// blocks; the slices go to a workspace and are added in a fixed order.
// Accumulator element e of lane l is row 4e + l/16, column l%16 of its 16 x 16 tile.
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace rr {

typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int GM_BM = 64, GM_BN = 64, GM_BK = 16, GM_THREADS = 256;
constexpr int GM_EL = GM_BM * GM_BK / GM_THREADS;   // tile elements per thread per step
constexpr int GM_PAD = 2;

// op(A)[i][k] for the tile element handled by (idx, s): 8 elements per thread.
template <typename T, bool TR>
RR_DEV void gm_load(const T* __restrict__ A, int64_t lda, int64_t rows, int64_t K, int64_t r0,
                    int64_t k0, int t, double (&v)[GM_EL]) {
#pragma unroll
    for (int s = 0; s < GM_EL; ++s) {
        int i, k;
        if (!TR) { i = t & 63; k = (t >> 6) + 4 * s; }     // consecutive rows contiguous
        else     { k = t & 15; i = (t >> 4) + 16 * s; }    // consecutive k contiguous
        const int64_t gi = r0 + i, gk = k0 + k;
        double x = 0.0;
        if (gi < rows && gk < K) x = (double)(TR ? A[gk + gi * lda] : A[gi + gk * lda]);
        v[s] = x;
    }
}
template <bool TR>
RR_DEV void gm_store(double (*S)[GM_BM + GM_PAD], int t, const double (&v)[GM_EL]) {
#pragma unroll
    for (int s = 0; s < GM_EL; ++s) {
        int i, k;
        if (!TR) { i = t & 63; k = (t >> 6) + 4 * s; }
        else     { k = t & 15; i = (t >> 4) + 16 * s; }
        S[k][i] = v[s];
    }
}

template <typename TA, typename TB, bool TRA, bool TRB, bool SYM = false>
__global__ __launch_bounds__(GM_THREADS) void k_gemm_mfma(int64_t M, int64_t N, int64_t K,
                                                          const TA* __restrict__ A, int64_t lda,
                                                          const TB* __restrict__ B, int64_t ldb,
                                                          double* __restrict__ C, int64_t ldc,
                                                          double alpha, double beta, int64_t kchunk,
                                                          double* __restrict__ part, int64_t gn,
                                                          int64_t ntiles, int64_t nwork, int64_t per_xcd,
                                                          bool b_upper) {
    __shared__ double As[GM_BK][GM_BM + GM_PAD];
    __shared__ double Bs[GM_BK][GM_BN + GM_PAD];
    // XCD-aware order: workgroups go to the 8 XCDs round robin, so block b runs on
    // XCD b % 8; each XCD takes one contiguous range of (slice, tile) indices, and
    // tiles that share an A row slab (and, split over K, the same K slice) meet in
    // one L2.  Tile t = bx * gn + by (bx <= by only, enumerated by rows of the upper
    // triangle, for a symmetric product).
    const int64_t L = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (L >= nwork) return;   // padding of the grid to a multiple of 8
    const int64_t bz = L / ntiles, tile = L % ntiles;
    int64_t bx, by;
    if (SYM) {
        by = (int64_t)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
        while (by * (by + 1) / 2 > tile) --by;
        while ((by + 1) * (by + 2) / 2 <= tile) ++by;
        bx = tile - by * (by + 1) / 2;
    } else {
        bx = tile / gn;
        by = tile % gn;
    }
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t i0 = bx * GM_BM;
    const int64_t j0 = by * GM_BN;
    const int64_t kb = bz * kchunk;
    int64_t ke = std::min<int64_t>(kb + kchunk, K);
    // op(B) upper triangular (zeros stored below the diagonal): column block j0 needs
    // only k < j0 + GM_BN
    if (b_upper) ke = std::min<int64_t>(ke, j0 + GM_BN);

    f64x4_t acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4_t{0.0, 0.0, 0.0, 0.0};

    // op(B)[k][j] is op(B^T)[j][k]: load it with the transposed flag.  Two register
    // sets alternate between k steps, so a tile is loaded two steps before it is
    // stored to LDS (the load latency of a step alone is not covered).
    double ra0[GM_EL], rb0[GM_EL], ra1[GM_EL], rb1[GM_EL];
    if (kb < ke) {
        gm_load<TA, TRA>(A, lda, M, ke, i0, kb, t, ra0);
        gm_load<TB, !TRB>(B, ldb, N, ke, j0, kb, t, rb0);
    }
    if (kb + GM_BK < ke) {
        gm_load<TA, TRA>(A, lda, M, ke, i0, kb + GM_BK, t, ra1);
        gm_load<TB, !TRB>(B, ldb, N, ke, j0, kb + GM_BK, t, rb1);
    }
    auto step = [&](int64_t k0, double (&ra)[GM_EL], double (&rb)[GM_EL]) {
        gm_store<TRA>(As, t, ra);
        gm_store<!TRB>(Bs, t, rb);
        __syncthreads();
        if (k0 + 2 * GM_BK < ke) {
            gm_load<TA, TRA>(A, lda, M, ke, i0, k0 + 2 * GM_BK, t, ra);
            gm_load<TB, !TRB>(B, ldb, N, ke, j0, k0 + 2 * GM_BK, t, rb);
        }
#pragma unroll
        for (int kc = 0; kc < GM_BK; kc += 4) {
            double a[2], b[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) a[u] = As[kc + (lane >> 4)][wm * 32 + u * 16 + (lane & 15)];
#pragma unroll
            for (int v = 0; v < 2; ++v) b[v] = Bs[kc + (lane >> 4)][wn * 32 + v * 16 + (lane & 15)];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[v], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
    };
    for (int64_t k0 = kb; k0 < ke; k0 += 2 * GM_BK) {
        step(k0, ra0, rb0);
        if (k0 + GM_BK < ke) step(k0 + GM_BK, ra1, rb1);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int64_t gj = j0 + wn * 32 + v * 16 + (lane & 15);
            if (gj >= N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gi = i0 + wm * 32 + u * 16 + 4 * e + (lane >> 4);
                if (gi >= M) continue;
                if (part) {
                    part[bz * M * N + gi + gj * M] = acc[u][v][e];
                } else {
                    double o = alpha * acc[u][v][e];
                    if (beta != 0.0) o = fma(beta, C[gi + gj * ldc], o);
                    C[gi + gj * ldc] = o;
                }
            }
        }
    }
}

__global__ void k_gemm_mfma_reduce(int64_t M, int64_t N, int splits, const double* __restrict__ part,
                                   double* __restrict__ C, int64_t ldc, double alpha, double beta) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < splits; ++z) s += part[(int64_t)z * total + e];
        const int64_t i = e % M, j = e / M;
        double o = alpha * s;
        if (beta != 0.0) o = fma(beta, C[i + j * ldc], o);
        C[i + j * ldc] = o;
    }
}

template <typename TA, typename TB, bool TRA, bool TRB, bool SYM = false>
static void gm_run(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                   int64_t ldb, double* C, int64_t ldc, double alpha, double beta, double* ws,
                   size_t wsd, hipStream_t st, bool b_upper = false) {
    const int64_t gm = (M + GM_BM - 1) / GM_BM, gn = (N + GM_BN - 1) / GM_BN;
    const int64_t kblocks = (K + GM_BK - 1) / GM_BK;
    const int64_t tiles = SYM ? gm * (gm + 1) / 2 : gm * gn;   // tiles that do work
    int64_t splits = 1;
    const int64_t target = 1024;   // four blocks per compute unit
    if (tiles < target && kblocks >= 16) {
        // round down: one more slice than fits would leave a second, nearly empty
        // round of blocks as long as the first
        splits = std::min<int64_t>(std::max<int64_t>(target / tiles, 1), kblocks / 8);
        splits = std::min<int64_t>(splits, 64);
        while (splits > 1 && (size_t)(splits * M * N) > wsd) --splits;
        splits = std::max<int64_t>(splits, 1);
    }
    const int64_t kchunk = ((kblocks + splits - 1) / splits) * GM_BK;
    splits = (K + kchunk - 1) / kchunk;
    // one launch dimension (padded to a multiple of 8) carries (slice, tile)
    const int64_t work = tiles * splits;
    const int64_t per_xcd = (work + 7) / 8;
    dim3 grid((unsigned)(per_xcd * 8));
    double* part = splits > 1 ? ws : nullptr;
    k_gemm_mfma<TA, TB, TRA, TRB, SYM><<<grid, GM_THREADS, 0, st>>>(M, N, K, (const TA*)A, lda,
                                                               (const TB*)B, ldb, C, ldc, alpha,
                                                               beta, kchunk, part, gn, tiles, work,
                                                               per_xcd, b_upper);
    if (part) {
        const int64_t g = std::min<int64_t>((M * N + 255) / 256, 16384);
        k_gemm_mfma_reduce<<<(unsigned)g, 256, 0, st>>>(M, N, (int)splits, part, C, ldc, alpha, beta);
    }
}

// C[i, j] = C[j, i] for i > j: completes a product whose tiles on and above the
// diagonal were formed.
__global__ void k_mirror_upper(int64_t M, double* __restrict__ C, int64_t ldc) {
    const int64_t total = M * M;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % M, j = e / M;
        if (i > j) C[i + j * ldc] = C[j + i * ldc];
    }
}

template <typename TA, typename TB>
static void gm_tr(bool trA, bool trB, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                  const void* B, int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                  double* ws, size_t wsd, hipStream_t st) {
    if (!trA && !trB) gm_run<TA, TB, false, false>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    else if (!trA && trB) gm_run<TA, TB, false, true>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    else if (trA && !trB) gm_run<TA, TB, true, false>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    else gm_run<TA, TB, true, true>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
}

bool launch_gemm_ata(int64_t M, int64_t K, const double* A, int64_t lda, double* C, int64_t ldc,
                     double* ws, size_t wsd, hipStream_t st) {
    if (M < 32 || K < 16) return false;
    gm_run<double, double, true, false, true>(M, M, K, A, lda, A, lda, C, ldc, 1.0, 0.0, ws, wsd, st);
    const int64_t g = std::min<int64_t>((M * M + 255) / 256, 16384);
    k_mirror_upper<<<(unsigned)g, 256, 0, st>>>(M, C, ldc);
    return true;
}

bool launch_gemm_upper_b(bool trA, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                         const double* B, int64_t ldb, double* C, int64_t ldc, double* ws, size_t wsd,
                         hipStream_t st) {
    if (M < 32 || N < 32 || K < 16) return false;
    if (trA) gm_run<double, double, true, false>(M, N, K, A, lda, B, ldb, C, ldc, 1.0, 0.0, ws, wsd, st, true);
    else gm_run<double, double, false, false>(M, N, K, A, lda, B, ldb, C, ldc, 1.0, 0.0, ws, wsd, st, true);
    return true;
}

bool launch_gemm_mfma(int dta, bool trA, int dtb, bool trB, int64_t M, int64_t N, int64_t K,
                      const void* A, int64_t lda, const void* B, int64_t ldb, double* C,
                      int64_t ldc, double alpha, double beta, double* ws, size_t wsd,
                      hipStream_t st) {
    if ((dta != DT_F64 && dta != DT_F32) || (dtb != DT_F64 && dtb != DT_F32)) return false;
    if (M < 32 || N < 32 || K < 16) return false;
    if (dta == DT_F64) {
        if (dtb == DT_F64) gm_tr<double, double>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
        else gm_tr<double, float>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    } else {
        if (dtb == DT_F64) gm_tr<float, double>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
        else gm_tr<float, float>(trA, trB, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, ws, wsd, st);
    }
    return true;
}

}  // namespace rr
