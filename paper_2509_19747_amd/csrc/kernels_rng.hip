// Random test matrices of the method (Section 1.1 eq. testmatrix, Section 2):
// Gaussian Omega / Theta / power-iteration starts and the SRHT test matrix,
// generated on the device from the counter-based SplitMix64 stream.
#include "common.hpp"
#include "kernels.hpp"

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
    k_iota<<<grid_for(s), 256, 0, st>>>(perm_ws, s);
    k_fisher_yates<<<1, 64, 0, st>>>(perm_ws, s, n, l, seed, rows_out);
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

}  // namespace rr
