// Dense sketch on bf16 MFMA: Y = A Omega + mu Omega for a stored symmetric A held
// in bf16 (mixed-precision mode) and a bf16 test matrix, float32 accumulation.
//
// A is symmetric, so row i of A (the MFMA A-operand: 8 consecutive k per lane)
// is read as column i of the column-major bf16 copy -- contiguous 16-byte loads.
// Block: 512 threads = 8 waves in a 4 (rows) x 2 (columns) grid of 64 x 128 wave
// tiles (2 x 4 tiles of v_mfma_f32_32x32x16_bf16, which sustains close to the bf16
// peak where the 16x16x32 form reaches about half); block tile 256 x 256; k step
// 64 (four MFMA depths).  The A and Omega slices are staged in LDS with padded
// rows, double-buffered (one barrier per step); the next step's global loads are
// issued before the current step's MFMAs and stored into the other buffer after them.
// Grid: x = column block (fastest), y = row block.
// Accumulator element j of lane l is row 8*(j/4) + 4*(l/32) + (j%4), column l%32
// of its 32 x 32 tile.
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace rr {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
constexpr int DG_BM = 256, DG_BN = 256, DG_BK = 64, DG_THREADS = 512;
constexpr int DG_LD = DG_BK + 8;   // padded LDS row (bf16)
constexpr int DG_CH = DG_BK / 8;   // 16-byte chunks per row of a slice
constexpr int DG_LOADS = DG_BM * DG_CH / DG_THREADS;   // chunks per thread and slice

__global__ __launch_bounds__(DG_THREADS) void k_dense_gemm_bf16(
    int64_t n, int64_t m, const uint16_t* __restrict__ A, int64_t lda,
    const uint16_t* __restrict__ B, int64_t ldb, float mu, float* __restrict__ Y, int64_t ldy) {
    // two buffers per slice: step k computes from one while step k+1 is stored into the
    // other, so one barrier per step orders both
    __shared__ __attribute__((aligned(16))) uint16_t As[2][DG_BM * DG_LD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][DG_BN * DG_LD];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave & 3, wn = wave >> 2;
    // the column block varies fastest: the blocks of one row block run together and
    // read the same slices of A within a short window, so the last-level cache serves
    // all but the first (A is read from HBM about once instead of once per column block)
    const int64_t i0 = (int64_t)blockIdx.y * DG_BM;
    const int64_t c0 = (int64_t)blockIdx.x * DG_BN;
    const bool vec_a = (lda % 8) == 0, vec_b = (ldb % 8) == 0;

    f32x16_t acc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[u][v][j] = 0.0f;

    // chunk q of a 256 x DG_BK slice: row q / DG_CH, 8 k values at 8 (q % DG_CH)
    auto load_chunk = [&](const uint16_t* base, int64_t ld, int64_t lim_row, int64_t row0,
                          int64_t k0, int q, bool vec) -> uint4 {
        const int r = q / DG_CH, part = q % DG_CH;
        const int64_t gr = row0 + r, gk = k0 + 8 * part;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gr < lim_row) {
            const uint16_t* src = base + gr * ld + gk;
            if (vec && gk + 8 <= n) {
                v = *(const uint4*)src;
            } else {
                uint32_t w[4] = {0u, 0u, 0u, 0u};
                for (int e = 0; e < 8; ++e)
                    if (gk + e < n) w[e >> 1] |= (uint32_t)src[e] << (16 * (e & 1));
                v = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
        return v;
    };

    uint4 ra[DG_LOADS], rb[DG_LOADS];
#pragma unroll
    for (int s = 0; s < DG_LOADS; ++s) {
        ra[s] = load_chunk(A, lda, n, i0, 0, t + DG_THREADS * s, vec_a);
        rb[s] = load_chunk(B, ldb, m, c0, 0, t + DG_THREADS * s, vec_b);
    }
    auto store = [&](int buf) {
#pragma unroll
        for (int s = 0; s < DG_LOADS; ++s) {
            const int q = t + DG_THREADS * s;
            *(uint4*)&As[buf][(q / DG_CH) * DG_LD + 8 * (q % DG_CH)] = ra[s];
            *(uint4*)&Bs[buf][(q / DG_CH) * DG_LD + 8 * (q % DG_CH)] = rb[s];
        }
    };
    store(0);
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = 0; k0 < n; k0 += DG_BK) {
        const bool more = k0 + DG_BK < n;
        if (more) {
#pragma unroll
            for (int s = 0; s < DG_LOADS; ++s) {
                ra[s] = load_chunk(A, lda, n, i0, k0 + DG_BK, t + DG_THREADS * s, vec_a);
                rb[s] = load_chunk(B, ldb, m, c0, k0 + DG_BK, t + DG_THREADS * s, vec_b);
            }
        }
        const int kq = 8 * (lane >> 5);
#pragma unroll
        for (int kh = 0; kh < DG_BK / 16; ++kh) {
            __builtin_amdgcn_sched_barrier(0);
            bf16x8_t a[2], b[4];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int row = wm * 64 + u * 32 + (lane & 31);
                a[u] = __builtin_bit_cast(bf16x8_t, *(const uint4*)&As[cur][row * DG_LD + 16 * kh + kq]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = wn * 128 + v * 32 + (lane & 31);
                b[v] = __builtin_bit_cast(bf16x8_t, *(const uint4*)&Bs[cur][col * DG_LD + 16 * kh + kq]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[u][v] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[u], b[v], acc[u][v], 0, 0, 0);
        }
        // the other buffer was last read before the previous barrier
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t gc = c0 + wn * 128 + v * 32 + (lane & 31);
            if (gc >= m) continue;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t gr = i0 + wm * 64 + u * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
                if (gr < n) {
                    const float bval = __uint_as_float((uint32_t)B[gc * ldb + gr] << 16);
                    Y[gr + gc * ldy] = fmaf(mu, bval, acc[u][v][j]);
                }
            }
        }
    }
}

void launch_dense_gemm_bf16(int64_t n, int64_t m, const void* A, int64_t lda, const void* B,
                            int64_t ldb, double mu, float* Y, int64_t ldy, hipStream_t st) {
    dim3 grid((unsigned)((m + DG_BN - 1) / DG_BN), (unsigned)((n + DG_BM - 1) / DG_BM));
    ProfScope prof(PROF_DENSE_SKETCH, st);
    k_dense_gemm_bf16<<<grid, DG_THREADS, 0, st>>>(n, m, (const uint16_t*)A, lda, (const uint16_t*)B,
                                                   ldb, (float)mu, Y, ldy);
}

}  // namespace rr
