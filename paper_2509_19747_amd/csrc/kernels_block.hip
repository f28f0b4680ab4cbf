// Small kernels of the block Krylov solvers (block preconditioned MINRES and block
// CG over s <= 32 right-hand sides under one shift, Section 7.2.2).
//
//  k_blk_chol   S (s x s, symmetrised) = C^T C with C upper; C^{-1}; a breakdown flag
//               when a pivot fails the rank rule c_jj^2 > 1e-20 S_jj (C and C^{-1}
//               are then zero, so products with them vanish).
//  k_bmr_qr     one step of the block QR of the band matrix T_k of block MINRES:
//               the new column block [C_k^T; M_k; C_{k+1}] takes the two previous
//               orthogonal factors, then a Householder QR of its last 2s x s part
//               gives R_kk and the next factor G_k (explicit 2s x 2s); the rotated
//               right-hand side [phi_k; phibar_{k+1}] = G_k^T [phibar_k; 0].
//  k_bmr_rows   the direction and solution updates, one thread per row:
//               D_k = (Z_k - D_{k-1} R_{k-1,k} - D_{k-2} R_{k-2,k}) R_kk^{-1}, the
//               same for A_mu D_k from A_mu Z_k, Y += D_k phi_k, R -= A_mu D_k phi_k.
//  k_blk_gather / k_blk_scatter  the columns of a cycle's block.
// All small matrices are column-major with leading dimension s.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rr {

constexpr int BLK_THREADS = 256;

__global__ __launch_bounds__(BLK_THREADS) void k_blk_chol(int s, const double* __restrict__ S,
                                                          double* __restrict__ C, double* __restrict__ Ci,
                                                          int32_t* __restrict__ flag) {
    __shared__ double a[BLOCK_MAX_S * BLOCK_MAX_S];
    __shared__ double ci[BLOCK_MAX_S * BLOCK_MAX_S];
    __shared__ double diag0[BLOCK_MAX_S];
    __shared__ int bad;
    const int t = threadIdx.x;
    for (int e = t; e < s * s; e += BLK_THREADS) {
        const int i = e % s, j = e / s;
        a[e] = 0.5 * (S[i + j * s] + S[j + i * s]);
        ci[e] = 0.0;
    }
    if (t == 0) bad = 0;
    __syncthreads();
    if (t < s) diag0[t] = a[t + t * s];
    __syncthreads();
    // right-looking Cholesky: row j of C from the trailing block, then its update
    for (int j = 0; j < s; ++j) {
        if (t == 0) {
            const double piv = a[j + j * s];
            if (!(diag0[j] > 0.0) || !(piv > 1e-20 * diag0[j])) bad = 1;
            else a[j + j * s] = sqrt(piv);
        }
        __syncthreads();
        if (bad) break;
        const double cjj = a[j + j * s];
        for (int k = j + 1 + t; k < s; k += BLK_THREADS) a[j + k * s] /= cjj;
        __syncthreads();
        for (int e = t; e < s * s; e += BLK_THREADS) {
            const int i = e % s, k = e / s;
            if (i > j && k >= i) a[i + k * s] -= a[j + i * s] * a[j + k * s];
        }
        __syncthreads();
    }
    if (bad) {
        for (int e = t; e < s * s; e += BLK_THREADS) { C[e] = 0.0; Ci[e] = 0.0; }
        if (t == 0) *flag = 1;
        return;
    }
    // C^{-1} column by column (thread j solves C x = e_j by back substitution)
    if (t < s) {
        const int j = t;
        for (int i = j; i >= 0; --i) {
            double v = (i == j) ? 1.0 : 0.0;
            for (int k = i + 1; k <= j; ++k) v -= a[i + k * s] * ci[k + j * s];
            ci[i + j * s] = v / a[i + i * s];
        }
    }
    __syncthreads();
    for (int e = t; e < s * s; e += BLK_THREADS) {
        const int i = e % s, k = e / s;
        C[e] = i <= k ? a[e] : 0.0;
        Ci[e] = i <= k ? ci[e] : 0.0;
    }
}

// X4: the column block k of T_k in rows of block rows k-2, k-1, k, k+1 (4s x s,
// leading dimension 4s).  G slots: G_{k-2}, G_{k-1} in, G_k out (2s x 2s each).
__global__ __launch_bounds__(BLK_THREADS) void k_bmr_qr(int s, int k, const double* __restrict__ M,
                                                        const double* __restrict__ Cprev,
                                                        const double* __restrict__ Cnew,
                                                        const int32_t* __restrict__ brk,
                                                        const double* __restrict__ Gm2,
                                                        const double* __restrict__ Gm1,
                                                        double* __restrict__ Gk, double* __restrict__ phibar,
                                                        double* __restrict__ R2, double* __restrict__ R1,
                                                        double* __restrict__ Rinv, double* __restrict__ phi) {
    constexpr int MS = BLOCK_MAX_S;
    __shared__ double X4[4 * MS * MS];
    __shared__ double G[4 * MS * MS];
    __shared__ double v[2 * MS];
    __shared__ double tmp[2 * MS * MS];
    __shared__ double red[BLK_THREADS];
    const int t = threadIdx.x;
    const int L = 4 * s, s2 = 2 * s;
    const bool broken = *brk != 0;
    for (int e = t; e < L * s; e += BLK_THREADS) {
        const int r = e % L, c = e / L;
        double x = 0.0;
        if (r >= s && r < 2 * s) x = k >= 1 ? Cprev[c + (r - s) * s] : 0.0;            // C_k^T
        else if (r >= 2 * s && r < 3 * s) x = M[(r - 2 * s) + c * s];
        else if (r >= 3 * s) x = broken ? 0.0 : Cnew[(r - 3 * s) + c * s];
        X4[r + c * L] = x;
    }
    __syncthreads();
    // previous factors: rows (k-2, k-1) by G_{k-2}^T, then rows (k-1, k) by G_{k-1}^T
    for (int pass = 0; pass < 2; ++pass) {
        const double* Gp = pass == 0 ? Gm2 : Gm1;
        if ((pass == 0 && k < 2) || (pass == 1 && k < 1)) continue;
        const int r0 = pass == 0 ? 0 : s;
        for (int e = t; e < s2 * s; e += BLK_THREADS) {
            const int i = e % s2, c = e / s2;
            double acc = 0.0;
            for (int r = 0; r < s2; ++r) acc += Gp[r + i * s2] * X4[r0 + r + c * L];
            tmp[e] = acc;
        }
        __syncthreads();
        for (int e = t; e < s2 * s; e += BLK_THREADS) {
            const int i = e % s2, c = e / s2;
            X4[r0 + i + c * L] = tmp[e];
        }
        __syncthreads();
    }
    // Householder QR of rows 2s..4s-1; G = H_0 H_1 ... H_{s-1}
    for (int e = t; e < s2 * s2; e += BLK_THREADS) G[e] = (e % s2 == e / s2) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = 0; j < s; ++j) {
        // v = x - alpha e_1 over rows j..2s-1 of the 2s-row part, alpha = -sign(x_0) ||x||
        double part = 0.0;
        for (int r = j + t; r < s2; r += BLK_THREADS) {
            const double x = X4[2 * s + r + j * L];
            part += x * x;
        }
        red[t] = part;
        __syncthreads();
        for (int w = BLK_THREADS / 2; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        // every thread reads the sum before the barrier that lets red be reused
        const double ss = red[0];
        const double x0 = X4[2 * s + j + j * L];
        __syncthreads();
        if (ss == 0.0) continue;
        const double nx = sqrt(ss);
        const double alpha = x0 >= 0.0 ? -nx : nx;
        for (int r = t; r < s2; r += BLK_THREADS)
            v[r] = r < j ? 0.0 : (r == j ? x0 - alpha : X4[2 * s + r + j * L]);
        __syncthreads();
        // v^T v = ||x||^2 - x0^2 + (x0 - alpha)^2 > 0, since |x0 - alpha| = |x0| + ||x||
        const double f = 2.0 / (ss - x0 * x0 + (x0 - alpha) * (x0 - alpha));
        // columns j..s-1 of the 2s-row part: x <- x - f v (v^T x)
        for (int c = j + t; c < s; c += BLK_THREADS) {
            double dv = 0.0;
            for (int r = j; r < s2; ++r) dv += v[r] * X4[2 * s + r + c * L];
            tmp[c] = dv;
        }
        // G <- G H_j: rows of G, g <- g - f (g v) v^T
        for (int r = t; r < s2; r += BLK_THREADS) {
            double gv = 0.0;
            for (int q = j; q < s2; ++q) gv += G[r + q * s2] * v[q];
            tmp[MS + r] = gv;
        }
        __syncthreads();
        for (int e = t; e < s2 * s; e += BLK_THREADS) {
            const int r = e % s2, c = e / s2;
            if (c >= j && r >= j) X4[2 * s + r + c * L] -= f * v[r] * tmp[c];
        }
        for (int e = t; e < s2 * s2; e += BLK_THREADS) {
            const int r = e % s2, q = e / s2;
            if (q >= j) G[r + q * s2] -= f * tmp[MS + r] * v[q];
        }
        __syncthreads();
    }
    for (int e = t; e < s2 * s2; e += BLK_THREADS) Gk[e] = G[e];
    // rotated right-hand side: phi = G[0:s,0:s]^T phibar, phibar' = G[0:s,s:2s]^T phibar
    for (int e = t; e < s * s; e += BLK_THREADS) {
        const int i = e % s, c = e / s;
        double a0 = 0.0, a1 = 0.0;
        for (int r = 0; r < s; ++r) {
            const double pb = phibar[r + c * s];
            a0 += G[r + i * s2] * pb;
            a1 += G[r + (s + i) * s2] * pb;
        }
        tmp[e] = a0;
        tmp[MS * MS + e] = a1;
    }
    __syncthreads();
    for (int e = t; e < s * s; e += BLK_THREADS) {
        phi[e] = tmp[e];
        phibar[e] = tmp[MS * MS + e];
        const int i = e % s, c = e / s;
        R2[e] = X4[i + c * L];
        R1[e] = X4[s + i + c * L];
    }
    // R_kk^{-1} (upper), thread j solves R x = e_j
    if (t < s) {
        const int j = t;
        for (int i = j; i >= 0; --i) {
            double acc = (i == j) ? 1.0 : 0.0;
            for (int q = i + 1; q <= j; ++q) acc -= X4[2 * s + i + q * L] * Rinv[q + j * s];
            Rinv[i + j * s] = acc / X4[2 * s + i + i * L];
        }
        for (int i = j + 1; i < s; ++i) Rinv[i + j * s] = 0.0;
    }
}

// out = (in - P1 R1 - P2 R2) Ri for one row held in registers (columns < s)
template <int MS>
__device__ __forceinline__ void blk_row(int64_t i, int64_t n, int s, const double* __restrict__ in,
                                        const double* __restrict__ P1, const double* __restrict__ P2,
                                        const double* R1, const double* R2, const double* Ri, double* o) {
    double tv[MS];
#pragma unroll
    for (int j = 0; j < MS; ++j) tv[j] = j < s ? in[i + (int64_t)j * n] : 0.0;
    for (int c = 0; c < s; ++c) {
        const double a = P1 ? P1[i + (int64_t)c * n] : 0.0;
        const double b = P2 ? P2[i + (int64_t)c * n] : 0.0;
#pragma unroll
        for (int j = 0; j < MS; ++j)
            if (j < s) tv[j] -= a * R1[c + j * s] + b * R2[c + j * s];
    }
#pragma unroll
    for (int j = 0; j < MS; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < MS; ++c)
            if (c <= j && j < s) acc += tv[c] * Ri[c + j * s];
        o[j] = acc;
    }
}

template <int MS>
__global__ __launch_bounds__(BLK_THREADS) void k_bmr_rows(int64_t n, int s, const double* __restrict__ Z,
                                                          const double* __restrict__ U,
                                                          const double* __restrict__ D1,
                                                          const double* __restrict__ D2,
                                                          const double* __restrict__ AD1,
                                                          const double* __restrict__ AD2,
                                                          const double* __restrict__ gR1,
                                                          const double* __restrict__ gR2,
                                                          const double* __restrict__ gRi,
                                                          const double* __restrict__ gphi, double* __restrict__ Dk,
                                                          double* __restrict__ ADk, double* __restrict__ Y,
                                                          double* __restrict__ Rres) {
    __shared__ double R1[MS * MS], R2[MS * MS], Ri[MS * MS], ph[MS * MS];
    for (int e = threadIdx.x; e < s * s; e += BLK_THREADS) {
        R1[e] = gR1[e]; R2[e] = gR2[e]; Ri[e] = gRi[e]; ph[e] = gphi[e];
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * BLK_THREADS + threadIdx.x;
    if (i >= n) return;
    double d[MS];
    blk_row<MS>(i, n, s, Z, D1, D2, R1, R2, Ri, d);
#pragma unroll
    for (int j = 0; j < MS; ++j)
        if (j < s) Dk[i + (int64_t)j * n] = d[j];
#pragma unroll
    for (int j = 0; j < MS; ++j) {
        if (j >= s) continue;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < MS; ++c)
            if (c < s) acc += d[c] * ph[c + j * s];
        Y[i + (int64_t)j * n] += acc;
    }
    blk_row<MS>(i, n, s, U, AD1, AD2, R1, R2, Ri, d);
#pragma unroll
    for (int j = 0; j < MS; ++j)
        if (j < s) ADk[i + (int64_t)j * n] = d[j];
#pragma unroll
    for (int j = 0; j < MS; ++j) {
        if (j >= s) continue;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < MS; ++c)
            if (c < s) acc += d[c] * ph[c + j * s];
        Rres[i + (int64_t)j * n] -= acc;
    }
}

__global__ void k_blk_gather(int64_t n, int s, const double* __restrict__ src, int64_t lds,
                             const int32_t* __restrict__ idx, double* __restrict__ dst) {
    const int64_t total = n * s;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, j = e / n;
        dst[e] = src[i + (int64_t)idx[j] * lds];
    }
}

__global__ void k_blk_scatter(int64_t n, int s, const double* __restrict__ src,
                              const int32_t* __restrict__ idx, double* __restrict__ dst, int64_t ldd, int add) {
    const int64_t total = n * s;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, j = e / n;
        double* o = dst + i + (int64_t)idx[j] * ldd;
        *o = add ? *o + src[e] : src[e];
    }
}

static unsigned blk_grid(int64_t work) {
    const int64_t g = (work + 255) / 256;
    return (unsigned)(g < 1 ? 1 : g > 65536 ? 65536 : g);
}

void launch_blk_chol(int s, const double* S, double* C, double* Ci, int32_t* flag, hipStream_t st) {
    k_blk_chol<<<1, BLK_THREADS, 0, st>>>(s, S, C, Ci, flag);
}

void launch_bmr_qr(int s, int k, const double* M, const double* Cprev, const double* Cnew, const int32_t* brk,
                   const double* Gm2, const double* Gm1, double* Gk, double* phibar, double* R2, double* R1,
                   double* Rinv, double* phi, hipStream_t st) {
    k_bmr_qr<<<1, BLK_THREADS, 0, st>>>(s, k, M, Cprev, Cnew, brk, Gm2, Gm1, Gk, phibar, R2, R1, Rinv, phi);
}

void launch_bmr_rows(int64_t n, int s, const double* Z, const double* U, const double* D1, const double* D2,
                     const double* AD1, const double* AD2, const double* R1, const double* R2,
                     const double* Rinv, const double* phi, double* Dk, double* ADk, double* Y, double* Rres,
                     hipStream_t st) {
    const unsigned g = (unsigned)((n + BLK_THREADS - 1) / BLK_THREADS);
#define BMR(MS) k_bmr_rows<MS><<<g, BLK_THREADS, 0, st>>>(n, s, Z, U, D1, D2, AD1, AD2, R1, R2, Rinv, phi, \
                                                          Dk, ADk, Y, Rres)
    if (s <= 8) BMR(8);
    else if (s <= 16) BMR(16);
    else BMR(32);
#undef BMR
}

void launch_blk_gather(int64_t n, int s, const double* src, int64_t lds, const int32_t* idx, double* dst,
                       hipStream_t st) {
    k_blk_gather<<<blk_grid(n * s), 256, 0, st>>>(n, s, src, lds, idx, dst);
}

void launch_blk_scatter(int64_t n, int s, const double* src, const int32_t* idx, double* dst, int64_t ldd,
                        bool add, hipStream_t st) {
    k_blk_scatter<<<blk_grid(n * s), 256, 0, st>>>(n, s, src, idx, dst, ldd, add ? 1 : 0);
}

}  // namespace rr
