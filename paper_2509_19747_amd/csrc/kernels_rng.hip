// Random test matrices of the method (Section 1.1 eq. testmatrix, Section 2):
// Gaussian Omega / Theta / power-iteration starts and the SRHT test matrix,
// generated on the device from the counter-based SplitMix64 stream.
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <climits>

namespace rr {

template <typename T>
__global__ void k_gauss_fill(T* __restrict__ out, int64_t rows, int64_t cols, int64_t ld,
                             uint64_t seed) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % rows, c = e / rows;
        out[i + c * ld] = from_f64<T>(gauss_at(seed, (uint64_t)e));
    }
}

__global__ void k_iota(int32_t* __restrict__ perm, int64_t s) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s;
         i += (int64_t)gridDim.x * blockDim.x)
        perm[i] = (int32_t)i;
}

// Partial Fisher-Yates over [0, s): l sequential swaps; step c swaps positions c
// and c + floor(hi32(word(n + c)) * (s - c) / 2^32).  One thread (l <= s is small).
__global__ void k_fisher_yates(int32_t* __restrict__ perm, int64_t s, int64_t n, int64_t l,
                               uint64_t seed, int32_t* __restrict__ rows_out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int64_t c = 0; c < l; ++c) {
        const uint64_t w = splitmix64(seed, (uint64_t)(n + c));
        const uint64_t span = (uint64_t)(s - c);
        const int64_t j = c + (int64_t)(((w >> 32) * span) >> 32);
        const int32_t t = perm[c];
        perm[c] = perm[j];
        perm[j] = t;
        rows_out[c] = perm[c];
    }
}

// The same shuffle with the permutation held in LDS as 16-bit entries (s <= 65536):
// the block fills it, then one thread makes the l swaps at LDS latency.
constexpr int FY_LDS_MAX = 65536;
__global__ __launch_bounds__(1024) void k_fisher_yates_lds(int64_t s, int64_t n, int64_t l, uint64_t seed,
                                                            int32_t* __restrict__ rows_out) {
    __shared__ uint16_t perm[FY_LDS_MAX];
    for (int64_t i = threadIdx.x; i < s; i += blockDim.x) perm[i] = (uint16_t)i;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int64_t c = 0; c < l; ++c) {
        const uint64_t w = splitmix64(seed, (uint64_t)(n + c));
        const uint64_t span = (uint64_t)(s - c);
        const int64_t j = c + (int64_t)(((w >> 32) * span) >> 32);
        const uint16_t t = perm[c];
        perm[c] = perm[j];
        perm[j] = t;
        rows_out[c] = (int32_t)perm[c];
    }
}

__global__ void k_srht_signs(float* __restrict__ D, int64_t n, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        D[i] = (splitmix64(seed, (uint64_t)i) >> 63) ? -1.0f : 1.0f;
}

// Omega[i, c] = D_i * (-1)^popcount(i & s_c): rows of the Sylvester Hadamard
// matrix sampled by s_c, signs D, restricted to the first n of s padded rows.
template <typename T>
__global__ void k_srht_fill(T* __restrict__ out, int64_t n, int64_t l, int64_t ld,
                            const float* __restrict__ D, const int32_t* __restrict__ rows) {
    const int64_t total = n * l;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, c = e / n;
        const int par = __popcll((unsigned long long)(i & (int64_t)rows[c])) & 1;
        const float v = par ? -D[i] : D[i];
        out[i + c * ld] = from_f64<T>((double)v);
    }
}

// Second-level sketch of Algorithm prec_chol_qr: S = Theta Y for the sparse sign
// embedding Theta (lsk = 2k rows, zeta = min(8, lsk) row blocks, block t = rows
// [floor(t lsk / zeta), floor((t+1) lsk / zeta))).  Column i of Theta has one entry
// per block t: word w of stream `seed` at counter i*zeta + t puts it at row
// r_t + floor(hi32(w) * b_t / 2^32) with sign -1 when bit 0 of w is set.
//   S[r, c] = sum over i (increasing) with row_t(i) = r of sign_t(i) Y[i, c],
// t the block that holds row r.  Y arrives row-major in float64 (Yt[i ldy + c]) so
// each hit adds one contiguous row.  One block per (row r, 256 columns): a pass
// hashes 2048 points, lists the hits of row r in LDS in increasing i (ballots in
// (slot, wave, lane) order), then adds their rows of Y in that order; the sum order
// is therefore fixed and equals the row order of Theta's CSR form.
constexpr int TH_THREADS = 256, TH_SLOTS = 8, TH_WAVES = TH_THREADS / WAVE;

__global__ __launch_bounds__(TH_THREADS) void k_theta_apply(int64_t n, int64_t k, int64_t lsk, int zeta,
                                                            uint64_t seed, const double* __restrict__ Yt,
                                                            int64_t ldy, double* __restrict__ S, int64_t lds,
                                                            int64_t row0, int accumulate) {
    __shared__ uint64_t bal[TH_SLOTS][TH_WAVES];
    __shared__ int32_t list[TH_SLOTS * TH_THREADS];
    const int64_t r = blockIdx.x;
    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
    int blk = 0;
    while (blk + 1 < zeta && (int64_t)(blk + 1) * lsk / zeta <= r) ++blk;
    const int64_t b0 = (int64_t)blk * lsk / zeta;
    const uint64_t bs = (uint64_t)((int64_t)(blk + 1) * lsk / zeta - b0);
    const int64_t c = (int64_t)blockIdx.y * TH_THREADS + t;
    const uint64_t below = (1ull << lane) - 1ull;
    double acc = 0.0;
    for (int64_t i0 = 0; i0 < n; i0 += TH_SLOTS * TH_THREADS) {
        bool hit[TH_SLOTS], neg[TH_SLOTS];
#pragma unroll
        for (int s = 0; s < TH_SLOTS; ++s) {
            const int64_t i = i0 + s * TH_THREADS + t;
            hit[s] = false;
            neg[s] = false;
            if (i < n) {
                const uint64_t wd = splitmix64(seed, (uint64_t)(row0 + i) * (uint64_t)zeta + (uint64_t)blk);
                hit[s] = b0 + (int64_t)(((wd >> 32) * bs) >> 32) == r;
                neg[s] = (wd & 1ull) != 0;
            }
            const uint64_t b = __ballot(hit[s]);
            if (lane == 0) bal[s][w] = b;
        }
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int s = 0; s < TH_SLOTS; ++s) {
#pragma unroll
            for (int v = 0; v < TH_WAVES; ++v) {
                const uint64_t b = bal[s][v];
                if (v == w && hit[s]) {
                    const int32_t off = s * TH_THREADS + t;   // i - i0
                    list[total + __popcll(b & below)] = neg[s] ? (off | INT32_MIN) : off;
                }
                total += __popcll(b);
            }
        }
        __syncthreads();
        if (c < k) {
            int j = 0;
            for (; j + 4 <= total; j += 4) {
                int32_t e[4];
                double y[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) e[q] = list[j + q];
#pragma unroll
                for (int q = 0; q < 4; ++q) y[q] = Yt[(i0 + (e[q] & INT32_MAX)) * ldy + c];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc += e[q] < 0 ? -y[q] : y[q];
            }
            for (; j < total; ++j) {
                const int32_t e = list[j];
                const double y = Yt[(i0 + (e & INT32_MAX)) * ldy + c];
                acc += e < 0 ? -y : y;
            }
        }
        __syncthreads();
    }
    if (c < k) S[r + c * lds] = accumulate ? S[r + c * lds] + acc : acc;
}

__global__ void k_srht_dbits(int64_t n, const float* __restrict__ D, uint32_t* __restrict__ dbits) {
    const int64_t words = (n + 31) / 32;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
         w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t b = 0;
        for (int q = 0; q < 32; ++q) {
            const int64_t i = 32 * w + q;
            if (i < n && D[i] < 0.0f) b |= 1u << q;
        }
        dbits[w] = b;
    }
}

static int grid_for(int64_t total, int block = 256) {
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_gauss_fill(void* out, int dtype, int64_t rows, int64_t cols, int64_t ld,
                       uint64_t seed, hipStream_t st) {
    const int g = grid_for(rows * cols);
    switch (dtype) {
        case DT_F64: k_gauss_fill<double><<<g, 256, 0, st>>>((double*)out, rows, cols, ld, seed); break;
        case DT_F32: k_gauss_fill<float><<<g, 256, 0, st>>>((float*)out, rows, cols, ld, seed); break;
        default: k_gauss_fill<__hip_bfloat16><<<g, 256, 0, st>>>((__hip_bfloat16*)out, rows, cols, ld, seed); break;
    }
}

void launch_srht_prepare(int64_t n, int64_t l, uint64_t seed, int64_t s, int32_t* perm_ws,
                         int32_t* rows_out, float* D_out, hipStream_t st) {
    if (s <= FY_LDS_MAX) {
        k_fisher_yates_lds<<<1, 1024, 0, st>>>(s, n, l, seed, rows_out);
    } else {
        k_iota<<<grid_for(s), 256, 0, st>>>(perm_ws, s);
        k_fisher_yates<<<1, 64, 0, st>>>(perm_ws, s, n, l, seed, rows_out);
    }
    k_srht_signs<<<grid_for(n), 256, 0, st>>>(D_out, n, seed);
}

void launch_srht_fill(void* out, int dtype, int64_t n, int64_t l, int64_t ld, const float* D,
                      const int32_t* rows, hipStream_t st) {
    const int g = grid_for(n * l);
    switch (dtype) {
        case DT_F64: k_srht_fill<double><<<g, 256, 0, st>>>((double*)out, n, l, ld, D, rows); break;
        case DT_F32: k_srht_fill<float><<<g, 256, 0, st>>>((float*)out, n, l, ld, D, rows); break;
        default: k_srht_fill<__hip_bfloat16><<<g, 256, 0, st>>>((__hip_bfloat16*)out, n, l, ld, D, rows); break;
    }
}

int theta_nnz(int64_t k) { return (int)std::min<int64_t>(THETA_NNZ, 2 * k); }

void launch_theta_apply(int64_t n, int64_t k, uint64_t seed, const double* Yt, int64_t ldy, double* S,
                        int64_t lds, hipStream_t st) {
    const int64_t lsk = 2 * k;
    dim3 grid((unsigned)lsk, (unsigned)((k + TH_THREADS - 1) / TH_THREADS));
    k_theta_apply<<<grid, TH_THREADS, 0, st>>>(n, k, lsk, theta_nnz(k), seed, Yt, ldy, S, lds, 0, 0);
}

void launch_theta_apply_rows(int64_t rows, int64_t row0, int64_t k, uint64_t seed, const double* Yt, int64_t ldy,
                             double* S, int64_t lds, bool accumulate, hipStream_t st) {
    const int64_t lsk = 2 * k;
    dim3 grid((unsigned)lsk, (unsigned)((k + TH_THREADS - 1) / TH_THREADS));
    k_theta_apply<<<grid, TH_THREADS, 0, st>>>(rows, k, lsk, theta_nnz(k), seed, Yt, ldy, S, lds, row0,
                                                accumulate ? 1 : 0);
}

void launch_srht_dbits(int64_t n, const float* D, uint32_t* dbits, hipStream_t st) {
    const int64_t words = (n + 31) / 32;
    k_srht_dbits<<<grid_for(words), 256, 0, st>>>(n, D, dbits);
}

// ------------------------------------------------ Y^T Omega for an SRHT Omega
// (Y^T Omega)[c, c'] = sum_i Y[i, c] D_i (-1)^popcount(i & s_c') is entry s_c' of the
// Walsh-Hadamard transform of D o Y[:, c] (length s, the power of two of the SRHT,
// zero past n).  With s = nch * ch and i = j ch + e, the transform factors into one
// of length ch per chunk j and a sum over the chunks with signs (-1)^popcount(j & s_hi):
// one pass transforms every nonzero chunk of every column in LDS, a second forms the
// l x l entries from the chunk transforms (16 chunk values each at n = 50,000).
constexpr int FW_THREADS = 256, FW_MAX = 4096;

template <typename T>
__global__ __launch_bounds__(FW_THREADS) void k_srht_fwht_chunks(int64_t n, int64_t ch, int nch,
                                                                 const T* __restrict__ Y, int64_t ldy,
                                                                 const uint32_t* __restrict__ dbits,
                                                                 double* __restrict__ W) {
    __shared__ double buf[FW_MAX];
    const int64_t c = blockIdx.y, j = blockIdx.x, base = j * ch;
    const int t = threadIdx.x;
    for (int64_t e = t; e < ch; e += FW_THREADS) {
        const int64_t i = base + e;
        double v = 0.0;
        if (i < n) {
            v = (double)Y[i + c * ldy];
            if ((dbits[i >> 5] >> (i & 31)) & 1u) v = -v;
        }
        buf[e] = v;
    }
    __syncthreads();
    for (int64_t h = 1; h < ch; h <<= 1) {
        for (int64_t q = t; q < ch / 2; q += FW_THREADS) {
            const int64_t i0 = (q / h) * 2 * h + (q % h);
            const double a = buf[i0], b = buf[i0 + h];
            buf[i0] = a + b;
            buf[i0 + h] = a - b;
        }
        __syncthreads();
    }
    double* out = W + (c * nch + j) * ch;
    for (int64_t e = t; e < ch; e += FW_THREADS) out[e] = buf[e];
}

// C[c + c' ldc] = sum_j (-1)^popcount(j & (s_c' / ch)) W[c, j, s_c' mod ch], chunks in order.
__global__ void k_srht_fwht_sample(int64_t l, int64_t ch, int nch, const double* __restrict__ W,
                                   const int32_t* __restrict__ rows, double* __restrict__ C, int64_t ldc) {
    const int64_t total = l * l;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e % l, cp = e / l;
        const int64_t sr = rows[cp];
        const int64_t hi = sr / ch, lo = sr % ch;
        const double* w = W + c * nch * ch + lo;
        double acc = 0.0;
        for (int j = 0; j < nch; ++j) {
            const double v = w[(int64_t)j * ch];
            acc += (__popcll((unsigned long long)(j & hi)) & 1) ? -v : v;
        }
        C[c + cp * ldc] = acc;
    }
}

int64_t srht_yt_omega_ws_doubles(int64_t n, int64_t l, int64_t s) {
    const int64_t ch = s < FW_MAX ? s : FW_MAX;
    return l * ((n + ch - 1) / ch) * ch;
}

void launch_srht_yt_omega(int ydt, int64_t n, int64_t l, int64_t s, const void* Y, int64_t ldy,
                          const uint32_t* dbits, const int32_t* rows, double* ws, double* C, int64_t ldc,
                          hipStream_t st) {
    const int64_t ch = s < FW_MAX ? s : FW_MAX;
    const int nch = (int)((n + ch - 1) / ch);   // chunks past n are zero
    const dim3 grid((unsigned)nch, (unsigned)l);
    if (ydt == DT_F32)
        k_srht_fwht_chunks<float><<<grid, FW_THREADS, 0, st>>>(n, ch, nch, (const float*)Y, ldy, dbits, ws);
    else
        k_srht_fwht_chunks<double><<<grid, FW_THREADS, 0, st>>>(n, ch, nch, (const double*)Y, ldy, dbits, ws);
    k_srht_fwht_sample<<<grid_for(l * l), 256, 0, st>>>(l, ch, nch, ws, rows, C, ldc);
}

}  // namespace rr
