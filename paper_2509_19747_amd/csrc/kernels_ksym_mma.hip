// Symmetric kernel matvec with the pair terms on bf16 MFMA:
// Y = scale * K U + mu U for NR = 1 or 2 columns (the PCG operator of kernel
// ridge regression, Section 7.2.2, and the two-column power iterations of the
// shift estimates).
//
// The exponent of each entry is the product of two augmented point records on
// bf16 MFMA, with float32-class accuracy (kmma.hpp).
//
// Rows are grouped in blocks of 256 (8 waves x 32 rows).  Work item (I, r, s)
// covers row block I against the column blocks J of run r (J = I + r m, ..., up to
// m of them, J < nb), restricted to the s-th of S column ranges.  Each pair (i, j)
// is evaluated once and its entry feeds y_i (row sums in registers) and y_j
// (column sums: the lane's 16 rows, then the two half-waves, then the eight waves
// in a fixed order): off the diagonal blocks by construction, and inside a
// diagonal block because wave w forms only the column tiles >= w and, in its own
// 32 x 32 tile, only the pairs with row <= column.  So the operator is exactly
// symmetric.
//
// Partial slots (float64, n per slot and column): the row sums of item (I, r, s) go
// to slot (I + r) S + s of the rows of I; column sums from row block I < J to slot
// I S of the columns (exactly one range s covers a column); column sums inside the
// diagonal block to slot nb S.  So row i of block b owns slots p S for p < b, the
// slots from b S to (b + R_b) S (R_b = ceil((nb - b) / m) runs) and slot nb S, each
// written by exactly one item, and the finish adds them in that order (bitwise
// reproducible).
//
#include "common.hpp"
#include "group.hpp"
#include "kentry.hpp"
#include "kernels.hpp"
#include "kmma.hpp"
#include "prof.hpp"

#include <algorithm>
#include <type_traits>

namespace rr {

constexpr int KM_WAVES = 8;
constexpr int KM_THREADS = 64 * KM_WAVES;
constexpr int KM_RB = 32 * KM_WAVES;   // rows (and columns) per block
constexpr int KM_CT = KM_RB / 32;      // column tiles per block
constexpr int KM_MAX_SLOTS = 2048;     // partial slots per row (bounds the workspace)

// Work items (I, r, s): row block I, run r of up to m column blocks starting at
// I + r m, column range s of S (S > 1 only with m = 1, for small n).
struct KmmaPlan {
    int nb, m, S;
    int64_t items;
};

static KmmaPlan kmma_plan(int64_t n) {
    KmmaPlan p;
    p.nb = (int)((n + KM_RB - 1) / KM_RB);
    const int64_t tiles = (int64_t)p.nb * (p.nb + 1) / 2;
    p.m = (int)std::min<int64_t>(8, std::max<int64_t>(1, tiles / 4096));
    int S = 1;
    while (p.m == 1 && S < KM_CT / 2 && tiles * S < 1024) S *= 2;   // a few items per compute unit
    p.S = S;
    int64_t runs = 0;
    for (int I = 0; I < p.nb; ++I) runs += (p.nb - I + p.m - 1) / p.m;
    p.items = runs * S;
    return p;
}

// Sum over the 32 lanes of a half-wave of v[0..15] (reduce-scatter butterfly in a
// fixed order): on return lanes 2e and 2e + 1 of the half hold the total of v[e].
template <typename T>
RR_DEV T kmma_rowsum16(T (&v)[16], int l32) {
    T w8[8], w4[4], w2[2];
    {
        const bool b = (l32 >> 4) & 1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const T keep = b ? v[8 + e] : v[e], send = b ? v[e] : v[8 + e];
            w8[e] = keep + __shfl_xor(send, 16, 64);
        }
    }
    {
        const bool b = (l32 >> 3) & 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const T keep = b ? w8[4 + e] : w8[e], send = b ? w8[e] : w8[4 + e];
            w4[e] = keep + __shfl_xor(send, 8, 64);
        }
    }
    {
        const bool b = (l32 >> 2) & 1;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const T keep = b ? w4[2 + e] : w4[e], send = b ? w4[e] : w4[2 + e];
            w2[e] = keep + __shfl_xor(send, 4, 64);
        }
    }
    const bool b = (l32 >> 1) & 1;
    const T keep = b ? w2[1] : w2[0], send = b ? w2[0] : w2[1];
    const T w1 = keep + __shfl_xor(send, 2, 64);
    // lanes 2e and 2e + 1 add the same two partials in opposite order: equal sums
    return w1 + __shfl_xor(w1, 1, 64);
}

// One work item of the block (see above).  T: the type of the products and partial
// sums (double; float for the estimate grade of the power iterations, whose per-item
// partials are still stored as double).  Shared by k_ksym_mma (item = block index)
// and the grouped serving kernel (items of many operators in one launch).
template <int KIND, int DM, int NR, typename T>
RR_DEV void ksym_mma_item(unsigned item, int64_t n, const float* __restrict__ xa, const float* __restrict__ sqn,
                          float c, const double* __restrict__ u, double* __restrict__ part, int nb, int m,
                          int S) {
    using Sh = KmmaShape<DM>;
    constexpr int KB = Sh::KB, BSTR = Sh::BSTR;
    __shared__ __attribute__((aligned(16))) __bf16 bs[KM_RB * BSTR];   // column records (B layout)
    __shared__ T us[NR][KM_RB];                                         // column u_j
    __shared__ __attribute__((aligned(16))) T ur[NR][KM_RB];            // row u_i
    __shared__ T colw[KM_WAVES][NR][KM_RB];                             // column partials per wave

    // item -> (bi, r, s)
    int64_t t = item / S;
    const int sr = (int)(item % S);
    int bi = 0;
    while (t >= (nb - bi + m - 1) / m) { t -= (nb - bi + m - 1) / m; ++bi; }
    const int run = (int)t;
    const int bj0 = bi + run * m, bj1 = std::min(bj0 + m, nb);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int64_t r0 = (int64_t)bi * KM_RB + 32 * wave;   // the wave's 32 rows
    const int cpr = KM_CT / S;                             // column tiles of a range
    const int ct0 = sr * cpr, ct1 = ct0 + cpr;
    const float g = KIND == 1 ? c : 1.0f;

    // the wave's rows: A operands, and u at the 16 rows of this lane's outputs
    bf16x8_t areg[KB];
    {
        const int64_t i = r0 + l32;
        const int64_t ic = i < n ? i : n - 1;
        kmma_record<DM, true>(xa + ic * DM, sqn[ic], g, h, [&](int s, const bf16x8_t& v) { areg[s] = v; });
    }
    T acc[16][NR];
#pragma unroll
    for (int e = 0; e < 16; ++e)
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[e][q] = T(0);
    for (int e = tid; e < NR * KM_RB; e += KM_THREADS) {
        const int q = e / KM_RB, rl = e % KM_RB;
        const int64_t i = (int64_t)bi * KM_RB + rl;
        ur[q][rl] = i < n ? T(u[(int64_t)q * n + i]) : T(0);
    }

    auto dots = [&](int ct) {
        const bf16x8_t* bp = reinterpret_cast<const bf16x8_t*>(&bs[(32 * ct + l32) * BSTR + 8 * h]);
        // B chunks two steps ahead of the MFMA that uses them
        bf16x8_t b0 = bp[0], b1 = KB > 1 ? bp[2] : b0;
        f32x16_t d;
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = 0.0f;
#pragma unroll
        for (int s = 0; s < KB; ++s) {
            const bf16x8_t b2 = s + 2 < KB ? bp[2 * (s + 2)] : b1;
            d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(areg[s], b0, d, 0, 0, 0);
            b0 = b1;
            b1 = b2;
        }
        return d;
    };
    // Columns past n carry u = 0 (no row-sum contribution; their column sums are
    // not stored); rows past n carry u = 0 likewise.
    // DG: the wave's own tile of a diagonal block; only pairs with row <= column
    // count (row sums), and row < column (column sums)
    auto entries = [&](int ct, const f32x16_t& dot, auto dg) {
        constexpr bool DG = decltype(dg)::value;
        const int jl = 32 * ct + l32;   // the lane's column within the block
        // u of the lane's rows, re-read from LDS for every tile (an opaque offset
        // keeps the compiler from holding all sixteen in registers)
        int uro = 32 * wave + 4 * h;
        asm volatile("" : "+v"(uro));
        T uj[NR], cs[2][NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            uj[q] = us[q][jl];
            cs[0][q] = T(0);
            cs[1][q] = T(0);
        }
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            // rows 8 g4 + 4 h + (0..3) of the wave: consecutive
            T ui[4][NR];
#pragma unroll
            for (int q = 0; q < NR; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) ui[r][q] = ur[q][uro + 8 * g4 + r];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = 4 * g4 + r;
                const T kv = T(kmma_entry<KIND>(dot[e], c));
                T kr = kv, kc = kv;
                if constexpr (DG) {
                    const int rr = 8 * g4 + 4 * h + r;   // the entry's row within the tile
                    kr = rr <= l32 ? kv : T(0);
                    kc = rr < l32 ? kv : T(0);
                }
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    acc[e][q] = fma(kr, uj[q], acc[e][q]);
                    cs[e & 1][q] = fma(kc, ui[r][q], cs[e & 1][q]);
                }
            }
        }
        // the two half-waves hold the same column for different rows; both store
        // the same sum (addition is commutative)
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const T v = cs[0][q] + cs[1][q];
            // (the lane swap for float64 sums; the float estimate-grade variant keeps the
            // permute, which spares it the swap's register copy at its register limit)
            if constexpr (sizeof(T) == 8) colw[wave][q][jl] = xor_pair_sum<32>(v);
            else colw[wave][q][jl] = v + __shfl_xor(v, 32, 64);
        }
    };

    const int64_t cslot = (int64_t)bi * S;
    const int64_t dslot = (int64_t)nb * S;   // column sums inside diagonal blocks
#pragma unroll 1
    for (int bj = bj0; bj < bj1; ++bj) {
        const int64_t cbase = (int64_t)bj * KM_RB;
        if (bj != bj0) __syncthreads();   // the previous block's records and partials are consumed
        // stage the column records: two threads per column, one per half of the
        // record chunks (columns past n: the last point, with u = 0)
        for (int e = tid; e < 2 * 32 * cpr; e += KM_THREADS) {
            const int jl = 32 * ct0 + (e >> 1), hh = e & 1;
            const int64_t j = cbase + jl;
            const int64_t jc = j < n ? j : n - 1;
            __bf16* dst = &bs[jl * BSTR + 8 * hh];
            kmma_record<DM, false>(xa + jc * DM, sqn[jc], g, hh, [&](int s, const bf16x8_t& v) {
                *reinterpret_cast<bf16x8_t*>(dst + 16 * s) = v;
            });
            if (hh == 0) {
#pragma unroll
                for (int q = 0; q < NR; ++q) us[q][jl] = j < n ? T(u[(int64_t)q * n + j]) : T(0);
            }
        }
        __syncthreads();
        // in the diagonal block wave w forms only the column tiles >= w, so each pair
        // is evaluated once and the operator stays exactly symmetric
        const int wlo = bj == bi ? wave : -1;
        if constexpr (NR == 2 && sizeof(T) == 8) {
            // Two columns with float64 sums: the next tile's exponent MFMAs are issued
            // before this tile's entries, so the matrix cores run while the vector ALU
            // works (the second accumulator fits this variant's registers; the others
            // would spill and run each tile's MFMAs and entries in turn, below).
            int ct = ct0;
            // in a diagonal block the tiles below the wave's own hold no pairs
            for (; ct < ct1 && ct < wlo; ++ct)
#pragma unroll
                for (int q = 0; q < NR; ++q) colw[wave][q][32 * ct + l32] = T(0);
            if (ct < ct1 && ct == wlo) {
                entries(ct, dots(ct), std::true_type{});
                ++ct;
            }
            if (ct < ct1) {
                f32x16_t dcur = dots(ct);
#pragma unroll 1
                for (; ct + 1 < ct1; ++ct) {
                    const f32x16_t dnext = dots(ct + 1);
                    __builtin_amdgcn_sched_barrier(0);
                    entries(ct, dcur, std::false_type{});
                    dcur = dnext;
                }
                entries(ct, dcur, std::false_type{});
            }
        } else {
#pragma unroll 1
            for (int ct = ct0; ct < ct1; ++ct) {
                if (ct <= wlo) {
                    if (ct == wlo) {
                        entries(ct, dots(ct), std::true_type{});
                    } else {
#pragma unroll
                        for (int q = 0; q < NR; ++q) colw[wave][q][32 * ct + l32] = T(0);
                    }
                    continue;
                }
                entries(ct, dots(ct), std::false_type{});
            }
        }
        __syncthreads();
        const int64_t slot = bj != bi ? cslot : dslot;
        for (int e = tid; e < NR * 32 * cpr; e += KM_THREADS) {
            const int q = e / (32 * cpr), jl = 32 * ct0 + e % (32 * cpr);
            const int64_t j = cbase + jl;
            if (j < n) {
                T v = T(0);
#pragma unroll
                for (int w = 0; w < KM_WAVES; ++w) v += colw[w][q][jl];
                part[(slot * NR + q) * n + j] = (double)v;
            }
        }
    }
    // row sums of the run
    const int64_t rslot = (int64_t)(bi + run) * S + sr;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        T v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = acc[e][q];
        const T tot = kmma_rowsum16(v, l32);
        const int e = l32 >> 1;
        const int64_t i = r0 + 8 * (e >> 2) + 4 * h + (e & 3);
        if ((l32 & 1) == 0 && i < n) part[(rslot * NR + q) * n + i] = (double)tot;
    }
}

template <int KIND, int DM, int NR, typename T>
__global__ __launch_bounds__(KM_THREADS) __attribute__((amdgpu_waves_per_eu(NR * sizeof(T) <= 8 ? 4 : 2))) void k_ksym_mma(
    int64_t n, const float* __restrict__ xa, const float* __restrict__ sqn, float c,
    const double* __restrict__ u, double* __restrict__ part, int nb, int m, int S,
    const int32_t* __restrict__ stop) {
    if (stop && *stop) return;
    ksym_mma_item<KIND, DM, NR, T>(blockIdx.x, n, xa, sqn, c, u, part, nb, m, S);
}

// y_q = scale * (sum of row i's slots) + mu u_q, with block partials of u_q^T y_q.
// Block: the 256 rows of one row block b (so the slot list is uniform over the
// block) and 1024 threads: four groups of 256 split the list
//   column slots p S (p < b), the run slots b S .. z1 - 1, the diagonal slot nb S
// into four contiguous quarters, each summed with four running sums, and group 0
// adds the quarters in a fixed order (bitwise reproducible, the same for one or
// two columns).
// Block bx of the nblk = ceil(n / 256) blocks of one finish (shared with the grouped
// serving kernel).
constexpr int KF_GROUPS = 4;
RR_DEV void ksym_mma_finish_block(unsigned bx, unsigned nblk, int64_t n, int rb, int nb, int m, int S, int nr,
                                  const double* __restrict__ part, double scale, double mu,
                                  const double* __restrict__ u, double* __restrict__ y,
                                  double* __restrict__ dot_part) {
    __shared__ double quart[KF_GROUPS - 1][256];
    __shared__ double sc[4];
    const int t = threadIdx.x & 255, g = threadIdx.x >> 8;
    const int64_t i = (int64_t)bx * 256 + t;
    const int b = (int)(((int64_t)bx * 256) / rb);
    const int64_t z1 = (int64_t)(b + (nb - b + m - 1) / m) * S;
    const int64_t nrun = z1 - (int64_t)b * S;
    const int64_t T = b + nrun + 1;
    const int64_t k0 = T * g / KF_GROUPS, k1 = T * (g + 1) / KF_GROUPS;
    auto slot = [&](int64_t k) -> int64_t {
        return k < b ? k * S : (k < b + nrun ? (int64_t)b * S + (k - b) : (int64_t)nb * S);
    };
    for (int q = 0; q < nr; ++q) {
        double s = 0.0;
        if (i < n) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            int64_t k = k0;
            for (; k + 4 <= k1; k += 4)
#pragma unroll
                for (int w = 0; w < 4; ++w) s4[w] += part[(slot(k + w) * nr + q) * n + i];
            for (; k < k1; ++k) s4[0] += part[(slot(k) * nr + q) * n + i];
            s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
        }
        // quart and sc are reused for the next column only after the barrier below
        if (g > 0) quart[g - 1][t] = s;
        __syncthreads();
        double dot = 0.0;
        if (g == 0 && i < n) {
            const double tot = (s + quart[0][t]) + (quart[1][t] + quart[2][t]);
            const double ui = u[(int64_t)q * n + i];
            const double yi = fma(scale, tot, mu * ui);
            y[(int64_t)q * n + i] = yi;
            dot = ui * yi;
        }
        if (g == 0) {
            dot = wave_sum(dot);
            if ((t & 63) == 0) sc[t >> 6] = dot;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            dot_part[(int64_t)q * nblk + bx] = (sc[0] + sc[1]) + (sc[2] + sc[3]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256 * KF_GROUPS) void k_ksym_mma_finish(int64_t n, int rb, int nb, int m, int S,
                                                                     int nr,
                                                                     const double* __restrict__ part,
                                                                     double scale, double mu,
                                                                     const double* __restrict__ u,
                                                                     double* __restrict__ y,
                                                                     double* __restrict__ dot_part,
                                                                     const int32_t* __restrict__ stop) {
    if (stop && *stop) return;
    ksym_mma_finish_block(blockIdx.x, gridDim.x, n, rb, nb, m, S, nr, part, scale, mu, u, y, dot_part);
}

// ------------------------------------------------------------------ float64
// The same work items, partial slots and finish as k_ksym_mma, with float64 entries
// (the restart residuals of the float64 refinement and the float64 working
// precision).  The Gram part of the exponent
//   t_ij = h_i + h_j + sum_k (g x_ik) x_jk = -g r_ij^2 / 2,   h_i = -g |x_i|^2 / 2,
// runs on v_mfma_f64_16x16x4_f64 with h_i as the accumulator's initial value; h_j,
// the table exp2 (kentry64) and the float64 row and column sums run on the vector
// ALU.  A wave's 32 x 32 tile is four 16 x 16 MFMA tiles (a, b): lane l supplies
// A[row 16 a + l%16][k 4 s + l/16] and B[k 4 s + l/16][column 16 b + l%16] of step s
// and holds element e of the product at row 16 a + 4 e + l/16, column 16 b + l%16, so
// a lane owns 8 rows and 2 columns of the tile.  Column sums: the lane's 8 rows, then
// the four lanes of a column (l/16 = 0..3), then the eight waves in a fixed order;
// row sums: the lane's columns over the item, then the 16 lanes of a row.  Each pair
// is evaluated once, also inside the diagonal blocks (wave w forms the column tiles
// >= w, and in its own tile only row <= column for the row sums and row < column for
// the column sums), so the operator is exactly symmetric.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <int KIND, int DM, int NR>
__global__ __launch_bounds__(KM_THREADS) __attribute__((amdgpu_waves_per_eu(NR == 1 ? 4 : 2))) void k_ksym_mma64(
    int64_t n, const double* __restrict__ xd, const double* __restrict__ hd, double g, double kconst,
    const double* __restrict__ u, double* __restrict__ part, int nb, int m, int S,
    const int32_t* __restrict__ stop) {
    constexpr int KS = DM / 4;   // MFMA steps of 4 coordinates
    __shared__ double bsd[DM][KM_RB];                 // column records, coordinate-major
    __shared__ double hs[KM_RB];                      // h_j
    __shared__ double hr[KM_RB];                      // h_i of the item's rows
    __shared__ double us[NR][KM_RB];                  // u_j
    __shared__ double colw[KM_WAVES][NR][KM_RB];      // column partials per wave
    __shared__ double tab[EXP2_TAB];
    if (stop && *stop) return;
    exp2_table_fill(tab);

    int64_t t = blockIdx.x / S;
    const int sr = (int)(blockIdx.x % S);
    int bi = 0;
    while (t >= (nb - bi + m - 1) / m) { t -= (nb - bi + m - 1) / m; ++bi; }
    const int run = (int)t;
    const int bj0 = bi + run * m, bj1 = std::min(bj0 + m, nb);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane >> 4, lc = lane & 15;
    const int64_t r0 = (int64_t)bi * KM_RB + 32 * wave;   // the wave's 32 rows
    const int cpr = KM_CT / S;
    const int ct0 = sr * cpr, ct1 = ct0 + cpr;

    // A operands (g x_i of rows 16 a + lc) and u_i at the lane's output rows; h_i of
    // the block's rows in LDS (read as the accumulators' initial values per tile)
    double areg[2][KS];
    double ui[8][NR], acc[8][NR];
    for (int e = tid; e < KM_RB; e += KM_THREADS) {
        const int64_t i = (int64_t)bi * KM_RB + e;
        hr[e] = hd[i < n ? i : n - 1];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int64_t i = r0 + 16 * a + lc;
        const int64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int s = 0; s < KS; ++s) areg[a][s] = g * xd[ic * DM + 4 * s + lr];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t ir = r0 + 16 * a + 4 * e + lr;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                ui[4 * a + e][q] = ir < n ? u[(int64_t)q * n + ir] : 0.0;
                acc[4 * a + e][q] = 0.0;
            }
        }
    }

    const int64_t cslot = (int64_t)bi * S;
    const int64_t dslot = (int64_t)nb * S;
#pragma unroll 1
    for (int bj = bj0; bj < bj1; ++bj) {
        const int64_t cbase = (int64_t)bj * KM_RB;
        __syncthreads();   // the previous block's records and partials are consumed (and the table is in)
        for (int e = tid; e < 32 * cpr; e += KM_THREADS) {
            const int jl = 32 * ct0 + e;
            const int64_t j = cbase + jl;
            const int64_t jc = j < n ? j : n - 1;
#pragma unroll
            for (int k = 0; k < DM; ++k) bsd[k][jl] = xd[jc * DM + k];
            hs[jl] = hd[jc];
#pragma unroll
            for (int q = 0; q < NR; ++q) us[q][jl] = j < n ? u[(int64_t)q * n + j] : 0.0;
        }
        __syncthreads();
        const int wlo = bj == bi ? wave : -1;
#pragma unroll 1
        for (int ct = ct0; ct < ct1; ++ct) {
            if (ct < wlo) {
                if (lr == 0)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int q = 0; q < NR; ++q) colw[wave][q][32 * ct + 16 * b + lc] = 0.0;
                continue;
            }
            auto tile = [&](auto dgc) {
                constexpr bool DG = decltype(dgc)::value;
                f64x4_t d[2][2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    f64x4_t h;
#pragma unroll
                    for (int e = 0; e < 4; ++e) h[e] = hr[32 * wave + 16 * a + 4 * e + lr];
                    d[a][0] = h;
                    d[a][1] = h;
                }
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const double b0 = bsd[4 * s + lr][32 * ct + lc];
                    const double b1 = bsd[4 * s + lr][32 * ct + 16 + lc];
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        d[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[a][s], b0, d[a][0], 0, 0, 0);
                        d[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[a][s], b1, d[a][1], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int jl = 32 * ct + 16 * b + lc;
                    const double hj = hs[jl];
                    double uj[NR], cs[NR];
#pragma unroll
                    for (int q = 0; q < NR; ++q) { uj[q] = us[q][jl]; cs[q] = 0.0; }
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const double kv = kentry64<KIND>(d[a][b][e] + hj, kconst, tab);
                            double kr = kv, kc = kv;
                            if constexpr (DG) {
                                const int rrow = 16 * a + 4 * e + lr, rcol = 16 * b + lc;
                                kr = rrow <= rcol ? kv : 0.0;
                                kc = rrow < rcol ? kv : 0.0;
                            }
#pragma unroll
                            for (int q = 0; q < NR; ++q) {
                                acc[4 * a + e][q] = fma(kr, uj[q], acc[4 * a + e][q]);
                                cs[q] = fma(kc, ui[4 * a + e][q], cs[q]);
                            }
                        }
                    // the four lanes of the column add in a fixed pattern (equal results)
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        double v = cs[q];
                        v = xor_pair_sum<16>(v);
                        v = xor_pair_sum<32>(v);
                        if (lr == 0) colw[wave][q][jl] = v;
                    }
                }
            };
            if (ct == wlo) tile(std::true_type{});
            else tile(std::false_type{});
        }
        __syncthreads();
        const int64_t slot = bj != bi ? cslot : dslot;
        for (int e = tid; e < NR * 32 * cpr; e += KM_THREADS) {
            const int q = e / (32 * cpr), jl = 32 * ct0 + e % (32 * cpr);
            const int64_t j = cbase + jl;
            if (j < n) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < KM_WAVES; ++w) v += colw[w][q][jl];
                part[(slot * NR + q) * n + j] = v;
            }
        }
    }
    // row sums of the run: the 16 lanes of a row add in a fixed butterfly
    const int64_t rslot = (int64_t)(bi + run) * S + sr;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            double v = acc[r][q];
            v = v + __shfl_xor(v, 1, 64);
            v = v + __shfl_xor(v, 2, 64);
            v = v + __shfl_xor(v, 4, 64);
            v = v + __shfl_xor(v, 8, 64);
            const int64_t i = r0 + 16 * (r >> 2) + 4 * (r & 3) + lr;
            if (lc == 0 && i < n) part[(rslot * NR + q) * n + i] = v;
        }
}

void launch_kernel_matvec_mma64(const KernelOp& op, const double* u, int nr, double mu, double* y,
                                double* dot_part, double* ws, const int32_t* stop, hipStream_t st) {
    const KmmaPlan p = kmma_plan(op.n);
    const double g = kernel_g64(op.kind, op.kconst);
    const unsigned grid = (unsigned)p.items;
    {
        ProfScope prof(nr == 1 ? PROF_KERNEL_MATVEC64 : -1, st);
#define KM64(K, DD, Q) k_ksym_mma64<K, DD, Q><<<grid, KM_THREADS, 0, st>>>(op.n, op.xd, op.hd, g, op.kconst, u, ws, p.nb, p.m, p.S, stop)
#define KM64D(K, Q)                      \
    switch (op.dm) {                     \
        case 4: KM64(K, 4, Q); break;    \
        case 8: KM64(K, 8, Q); break;    \
        case 16: KM64(K, 16, Q); break;  \
        default: KM64(K, 32, Q); break;  \
    }
        if (op.kind == 1) {
            if (nr == 1) { KM64D(1, 1) } else { KM64D(1, 2) }
        } else {
            if (nr == 1) { KM64D(2, 1) } else { KM64D(2, 2) }
        }
#undef KM64D
#undef KM64
    }
    k_ksym_mma_finish<<<(unsigned)((op.n + 255) / 256), 256 * KF_GROUPS, 0, st>>>(op.n, KM_RB, p.nb, p.m, p.S, nr, ws,
                                                                      op.scale, mu, u, y, dot_part,
                                                                      stop);
}

template <int KIND, int NR, typename T>
static void kmma_dispatch(const KernelOp& op, float c, const double* u, double* ws,
                          const KmmaPlan& p, const int32_t* stop, hipStream_t st) {
    const unsigned grid = (unsigned)p.items;
#define KML(DD)                                                                                    \
    k_ksym_mma<KIND, DD, NR, T><<<grid, KM_THREADS, 0, st>>>(op.n, op.xa, op.sqn, c, u, ws, p.nb, \
                                                             p.m, p.S, stop)
    switch (op.dm) {
        case 4: KML(4); break;
        case 8: KML(8); break;
        case 16: KML(16); break;
        default:
            // four columns of 32-term records exceed the LDS (callers use at most two)
            if constexpr (NR <= 2) KML(32);
            break;
    }
#undef KML
}

int kernel_mma_max_cols(int dm) { return dm <= 16 ? 4 : 2; }

bool kernel_mma_ok(int64_t n, int d) {
    const KmmaPlan p = kmma_plan(n);
    return d <= 32 && (int64_t)p.nb * p.S + 1 <= KM_MAX_SLOTS;
}

KmmaPlanInfo kernel_mma_plan_info(int64_t n) {
    const KmmaPlan p = kmma_plan(n);
    return KmmaPlanInfo{p.nb, p.m, p.S, p.items};
}

size_t kernel_mma_ws_doubles(int64_t n, int nr) {
    const KmmaPlan p = kmma_plan(n);
    return ((size_t)p.nb * p.S + 1) * nr * (size_t)n;
}

// nr in {1, 2} (also 4 with float64 sums when kernel_mma_max_cols(dm) allows); u, y
// column-major with leading dimension n; ws holds kernel_mma_ws_doubles(n, nr) doubles.
// a32: float32 products and partial sums (estimate grade, nr <= 2).
void launch_kernel_matvec_mma(const KernelOp& op, const double* u, int nr, double mu, double* y,
                              double* dot_part, double* ws, const int32_t* stop, hipStream_t st,
                              bool a32) {
    const KmmaPlan p = kmma_plan(op.n);
    const float c = kernel_c32(op.kind, op.kconst);
    {
        ProfScope prof(nr == 1 && !a32 ? PROF_KERNEL_MATVEC : -1, st);
#define KMD(K)                                                                   \
    if (a32) {                                                                   \
        if (nr == 1) kmma_dispatch<K, 1, float>(op, c, u, ws, p, stop, st);      \
        else kmma_dispatch<K, 2, float>(op, c, u, ws, p, stop, st);              \
    } else {                                                                     \
        if (nr == 1) kmma_dispatch<K, 1, double>(op, c, u, ws, p, stop, st);     \
        else if (nr == 2) kmma_dispatch<K, 2, double>(op, c, u, ws, p, stop, st); \
        else kmma_dispatch<K, 4, double>(op, c, u, ws, p, stop, st);             \
    }
        if (op.kind == 1) { KMD(1) } else { KMD(2) }
#undef KMD
    }
    k_ksym_mma_finish<<<(unsigned)((op.n + 255) / 256), 256 * KF_GROUPS, 0, st>>>(op.n, KM_RB, p.nb, p.m, p.S, nr, ws,
                                                                      op.scale, mu, u, y, dot_part,
                                                                      stop);
}

// ------------------------------------------------------------------ grouped
// The product and finish of many column blocks (of many requests) in one persistent
// launch each: work item w of the list belongs to the block whose first item is the
// largest <= w, and runs that block's item w - w_mat (the same block of threads
// k_ksym_mma would run for it).  Column blocks whose columns have all stopped are
// skipped.
RR_DEV bool group_pair_runs(const GPair& g) {
    const BState* st = gu(g.st);
    const int32_t nc = gu(g.ncols);
    for (int32_t q = 0; q < nc; ++q)
        if (gu(st[q].run)) return true;
    return false;
}

template <int KIND, int DM, int NR>
__global__ __launch_bounds__(KM_THREADS) __attribute__((amdgpu_waves_per_eu(NR == 1 ? 4 : 2))) void k_group_mat(
    const GTable* __restrict__ tab, int list, const GPair* __restrict__ units, int32_t* ctr) {
    __shared__ int32_t wsh;
    const int32_t off = gu(tab->list[list].off), cnt = gu(tab->list[list].count);
    const int32_t total = gu(tab->list[list].total);
    GroupCursor cur(ctr, &wsh);
    while (true) {
        const int32_t w = cur.next();
        if (w >= total) return;
        const int32_t ui = group_find(units, off, off + cnt, w, [](const GPair& g) { return g.w_mat; });
        const GPair& g = units[ui];
        if (!group_pair_runs(g)) continue;
        ksym_mma_item<KIND, DM, NR, double>((unsigned)(w - gu(g.w_mat)), gu(g.n), gu(g.xa), gu(g.sqn), gu(g.c),
                                            gu(g.u), gu(g.part), gu(g.nb), gu(g.m), gu(g.S));
    }
}

__global__ __launch_bounds__(256 * KF_GROUPS) void k_group_fin(const GTable* __restrict__ tab,
                                                               const GPair* __restrict__ units, int32_t* ctr) {
    __shared__ int32_t wsh;
    const int32_t off = gu(tab->list[GL_FIN].off), cnt = gu(tab->list[GL_FIN].count);
    const int32_t total = gu(tab->list[GL_FIN].total);
    GroupCursor cur(ctr, &wsh);
    while (true) {
        const int32_t w = cur.next();
        if (w >= total) return;
        const int32_t ui = group_find(units, off, off + cnt, w, [](const GPair& g) { return g.w_fin; });
        const GPair& g = units[ui];
        if (!group_pair_runs(g)) continue;
        ksym_mma_finish_block((unsigned)(w - gu(g.w_fin)), (unsigned)gu(g.nfb), gu(g.n), KM_RB, gu(g.nb),
                              gu(g.m), gu(g.S), gu(g.nr), gu(g.part), gu(g.scale), gu(g.mu), gu(g.u), gu(g.y),
                              gu(g.dot));
    }
}

int group_mat_list(int kind, int dm, int nr) {
    return GL_MAT + 12 * (kind - 1) + 3 * group_rec_class(dm) + (nr >= 4 ? 2 : nr >= 2 ? 1 : 0);
}

template <int KIND, int DM>
static void group_mat_width(int wc, int list, int blocks, const GTable* tab, const GPair* pairs, int32_t* ctr,
                            hipStream_t st) {
    if (wc == 0) k_group_mat<KIND, DM, 1><<<blocks, KM_THREADS, 0, st>>>(tab, list, pairs, ctr);
    else if (wc == 1) k_group_mat<KIND, DM, 2><<<blocks, KM_THREADS, 0, st>>>(tab, list, pairs, ctr);
    else if constexpr (DM <= 16) k_group_mat<KIND, DM, 4><<<blocks, KM_THREADS, 0, st>>>(tab, list, pairs, ctr);
}

void launch_group_mat(int list, int blocks, const GTable* tab, const GPair* pairs, int32_t* ctr, hipStream_t st) {
    const int kind = (list - GL_MAT) / 12 + 1, rc = ((list - GL_MAT) % 12) / 3, wc = (list - GL_MAT) % 3;
#define KGMD(K)                                                              \
    switch (rc) {                                                            \
        case 0: group_mat_width<K, 4>(wc, list, blocks, tab, pairs, ctr, st); break;   \
        case 1: group_mat_width<K, 8>(wc, list, blocks, tab, pairs, ctr, st); break;   \
        case 2: group_mat_width<K, 16>(wc, list, blocks, tab, pairs, ctr, st); break;  \
        default: group_mat_width<K, 32>(wc, list, blocks, tab, pairs, ctr, st); break; \
    }
    if (kind == 1) { KGMD(1) } else { KGMD(2) }
#undef KGMD
}

void launch_group_fin(int blocks, const GTable* tab, const GPair* pairs, int32_t* ctr, hipStream_t st) {
    k_group_fin<<<blocks, 256 * KF_GROUPS, 0, st>>>(tab, pairs, ctr);
}

}  // namespace rr
