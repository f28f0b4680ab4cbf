// Shared device/host utilities for the RandRAND gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>

#define RR_DEV __device__ __forceinline__

namespace rr {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ numerics
template <typename T> RR_DEV double to_f64(T v);
template <> RR_DEV double to_f64<double>(double v) { return v; }
template <> RR_DEV double to_f64<float>(float v) { return (double)v; }
template <> RR_DEV double to_f64<__hip_bfloat16>(__hip_bfloat16 v) { return (double)__bfloat162float(v); }

template <typename T> RR_DEV T from_f64(double v);
template <> RR_DEV double from_f64<double>(double v) { return v; }
template <> RR_DEV float from_f64<float>(double v) { return (float)v; }
template <> RR_DEV __hip_bfloat16 from_f64<__hip_bfloat16>(double v) {
    // round the float64 value to float32 first, then to bf16 with round-to-nearest-even
    // on the top 16 bits (finite inputs)
    const uint32_t u = __float_as_uint((float)v);
    const uint16_t b = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    return __builtin_bit_cast(__hip_bfloat16, b);
}

// ------------------------------------------------- deterministic reductions
// Wave-level sum with a fixed butterfly order: every lane gets the same result.
RR_DEV double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}
RR_DEV float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// v[l] + v[l ^ 32] (XOR = 32) or v[l] + v[l ^ 16] (XOR = 16) in every lane, the same value
// as v + __shfl_xor(v, XOR) (addition is commutative), with gfx950's lane-swap moves
// instead of an LDS permute.  A swap of a register with itself leaves the two
// partners of a lane in the two results, so their sum is the pair's sum.
template <int XOR>
RR_DEV uint2 lane_swap_pair(uint32_t u) {
    static_assert(XOR == 16 || XOR == 32, "lane_swap_pair: XOR must be 16 or 32");
    if constexpr (XOR == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        return make_uint2(r[0], r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        return make_uint2(r[0], r[1]);
    }
}
template <int XOR>
RR_DEV double xor_pair_sum(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint2 lo = lane_swap_pair<XOR>((uint32_t)b), hi = lane_swap_pair<XOR>((uint32_t)(b >> 32));
    const double x = __builtin_bit_cast(double, ((uint64_t)hi.x << 32) | lo.x);
    const double y = __builtin_bit_cast(double, ((uint64_t)hi.y << 32) | lo.y);
    return x + y;
}
template <int XOR>
RR_DEV float xor_pair_sum(float v) {
    const uint2 r = lane_swap_pair<XOR>(__builtin_bit_cast(uint32_t, v));
    return __builtin_bit_cast(float, r.x) + __builtin_bit_cast(float, r.y);
}

// DPP wave reduction towards lane 63.  One step on a float64 value (the same
// DPP move on both halves; rows outside row_mask read 0 and keep their value).
template <int CTRL, int ROWMASK>
RR_DEV double dpp_add(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWMASK, 0xF, false);
    return v + __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int CTRL, int ROWMASK>
RR_DEV float dpp_add(float v) {
    const int t = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWMASK, 0xF, false);
    return v + __builtin_bit_cast(float, t);
}
// Sum over the 64 lanes, valid in lane 63: pairs and quads (quad_perm), half
// rows (row_half_mirror), rows (row_mirror), then row 0 into 1 and 2 into 3
// (row_bcast:15), then rows 0-1 into 2-3 (row_bcast:31).
template <typename T, int M>
RR_DEV void wave_sum_to63(T (&v)[M]) {
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = dpp_add<0xB1, 0xF>(v[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = dpp_add<0x4E, 0xF>(v[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = dpp_add<0x141, 0xF>(v[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = dpp_add<0x140, 0xF>(v[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = dpp_add<0x142, 0xA>(v[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = dpp_add<0x143, 0xC>(v[m]);
}

// Block sum of one double per thread; result returned to every thread.
// `scratch` must hold blockDim.x/64 doubles.  Fixed order -> deterministic.
RR_DEV double block_sum(double v, double* scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
}

// Sum `count` doubles from global memory in a fixed order with one block.
RR_DEV double block_sum_array(const double* __restrict__ a, int count, double* scratch) {
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) v += a[i];
    return block_sum(v, scratch);
}

// -------------------------------------------------------- counter-based RNG
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): word k of the stream seeded
// with s is the 64-bit finaliser applied to s + (k+1) * 0x9E3779B97F4A7C15.
RR_DEV uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Box-Muller (cosine branch) from words 2e and 2e+1: u1 in (0,1], u2 in [0,1).
RR_DEV double gauss_at(uint64_t seed, uint64_t e) {
    const uint64_t w1 = splitmix64(seed, 2ull * e);
    const uint64_t w2 = splitmix64(seed, 2ull * e + 1ull);
    const double u1 = ((double)(w1 >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(w2 >> 11) * 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

}  // namespace rr
