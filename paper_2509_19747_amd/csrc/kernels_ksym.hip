// Symmetric float32 kernel matvec: Y = scale * K U + mu U for U with NR columns
// (the PCG operator of kernel ridge regression, Section 7.2.2, and the
// two-column power iterations of the tau estimates).
//
// K is symmetric, so every unordered pair of row blocks (I, J), I < J, is
// formed once: the block's threads own rows of I (coordinates in VGPRs), the
// points of J stream through scalar loads (wave-uniform), and each entry K_ij
// feeds both the row sum y_i += K_ij u_j and the column sum y_j += K_ij u_i.
// Diagonal blocks (I = J) form the full square and keep row sums only.
//
// Precision: float32 entries (bitwise symmetric, see kentry.hpp), widened to
// float64 for every product with u and every sum (row sums in registers,
// column sums over the thread's rows, a fixed DPP tree over the wave and the
// block's four waves).  Float32 accumulation would make the operator depend
// on u through rounding at the 1e-7 level, which caps the residual PCG can
// reach near 1e-7 * ||A|| ||x|| / ||b||; float64 keeps it a fixed linear map
// (the float32-rounded symmetric matrix).  Every partial lands in its own slot
// of the workspace and the finish kernel adds a row's slots in a fixed order,
// so results are bitwise reproducible.
//
// Work items: (I, J, s) for I <= J and s = 0..S-1, the s-th slice of CL
// columns of block J.  Row partials of item (I, J, s) go to slot J*S + s of
// the rows of I; column partials go to slot I*S of the columns of J (I < J,
// so these slots never meet a row slot of the same row, whose partner block
// is >= its own block).
#include "common.hpp"
#include "kentry.hpp"
#include "kernels.hpp"
#include "prof.hpp"

#include <algorithm>

namespace rr {

constexpr int KS_THREADS = 256;
// columns per LDS column-sum round (LDS: 4 waves x chunk x NR doubles = 16 KB)
constexpr int ks_chunk_ct(int NR) { return NR >= 8 ? 64 : NR >= 4 ? 128 : 256; }

// Points are read as zero-padded records of DM floats (DM = 4, 8, 16, 32):
// one scalar load brings a whole column point into SGPRs, and the padding adds
// exact zeros to the dot product.  Rows per thread and points per step shrink
// as DM and NR grow so that coordinates, accumulators and the step's scalar
// operands stay in registers.
constexpr int ksym_rows_ct(int DM, int NR, bool A32 = false) {
    // R * (DM + 4 NR) (float64 sums) or R * (DM + 3 NR) (float32 estimate) VGPRs
    return A32 ? (DM + 3 * NR <= 24 ? 8 : DM + 3 * NR <= 42 ? 4 : 2)
               : (DM + 4 * NR <= 21 ? 8 : DM + 4 * NR <= 42 ? 4 : 2);
}
constexpr int ksym_jb_ct(int DM, int NR) {
    const int base = DM <= 8 ? 4 : DM <= 16 ? 2 : 1;
    const int div = NR >= 8 ? 4 : NR >= 4 ? 2 : 1;
    return base / div > 0 ? base / div : 1;
}

struct KsymPlan {
    int R, RB, nb, S, CL;
    int64_t items;
};

static KsymPlan ksym_plan(int64_t n, int d, int nr, bool a32 = false) {
    KsymPlan p;
    p.R = ksym_rows_ct(kernel_record_len(d), nr, a32);
    p.RB = KS_THREADS * p.R;
    p.nb = (int)((n + p.RB - 1) / p.RB);
    const int64_t tiles = (int64_t)p.nb * (p.nb + 1) / 2;
    const int64_t target = nr >= 4 ? 1024 : 2048;
    int64_t S = (target + tiles - 1) / tiles;
    S = std::min<int64_t>(S, std::max(1, p.RB / 64));
    S = std::max<int64_t>(S, 1);
    p.S = (int)S;
    p.CL = (p.RB + p.S - 1) / p.S;
    p.items = tiles * p.S;
    return p;
}

size_t kernel_sym_ws_doubles(int64_t n, int d, int nr) {
    size_t w = 0;
    for (int a = 0; a < 2; ++a) {
        const KsymPlan p = ksym_plan(n, d, nr, a == 1);
        w = std::max(w, (size_t)p.nb * p.S * nr * (size_t)n);
    }
    return w;
}

// JB points [j, j + JB) of one item.  OFFD adds column sums.  A32: products
// and sums in float32 (an estimate-grade operator for the power iterations of
// the tau estimates; row sums still go to float64 every JB points).
template <bool A32> struct KsymT { typedef double U; };
template <> struct KsymT<true> { typedef float U; };

template <int KIND, int DM, int NR, int R, int JB, bool OFFD, bool A32>
RR_DEV void ksym_step(int64_t n, const float* __restrict__ xa, const float* __restrict__ sqn,
                      float c, const double* __restrict__ u, int64_t j, int64_t c0,
                      const float (&xi)[R][DM], const float (&mhn)[R],
                      const typename KsymT<A32>::U (&ui)[R][NR], double (&acc)[R][NR], double* colw,
                      int lane) {
    typedef typename KsymT<A32>::U U;
    U cp[JB * NR];
    float a32[R][NR];
    if constexpr (A32) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < NR; ++q) a32[r][q] = 0.0f;
    }
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
        const int64_t jj = j + jb;
        const float nj = sqn[jj];
        U uj[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) uj[q] = (U)u[(int64_t)q * n + jj];
        float s[R];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = kpair_init(mhn[r], nj);
        const float* xj = xa + jj * DM;
#pragma unroll
        for (int k = 0; k < DM; ++k) {
            const float xjk = xj[k];
#pragma unroll
            for (int r = 0; r < R; ++r) s[r] = fmaf(xi[r][k], xjk, s[r]);
        }
        U kv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) kv[r] = (U)kval32<KIND>(s[r], c);
        if constexpr (A32) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int q = 0; q < NR; ++q) a32[r][q] = fmaf(kv[r], uj[q], a32[r][q]);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int q = 0; q < NR; ++q) acc[r][q] = fma(kv[r], uj[q], acc[r][q]);
        }
        if (OFFD) {
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                U t = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) t = kv[r] * ui[r][q] + t;
                cp[jb * NR + q] = t;
            }
        }
    }
    if constexpr (A32) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[r][q] += (double)a32[r][q];
    }
    if (OFFD) {
        wave_sum_to63(cp);
        if (lane == 63) {
            const int base = (int)(j - c0) * NR;
#pragma unroll
            for (int m = 0; m < JB * NR; ++m) colw[base + m] = (double)cp[m];
        }
    }
}

template <int KIND, int DM, int NR, bool OFFD, bool A32>
RR_DEV void ksym_columns(int64_t n, const float* __restrict__ xa,
                         const float* __restrict__ sqn, float c, const double* __restrict__ u,
                         double* __restrict__ part, int64_t cb, int64_t ce, int64_t colslot,
                         const float (&xi)[ksym_rows_ct(DM, NR, A32)][DM],
                         const float (&mhn)[ksym_rows_ct(DM, NR, A32)],
                         const typename KsymT<A32>::U (&ui)[ksym_rows_ct(DM, NR, A32)][NR],
                         double (&acc)[ksym_rows_ct(DM, NR, A32)][NR],
                         double (*colw)[ks_chunk_ct(NR) * NR]) {
    constexpr int CH = ks_chunk_ct(NR);
    constexpr int R = ksym_rows_ct(DM, NR, A32);
    constexpr int JB = ksym_jb_ct(DM, NR);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t c0 = cb; c0 < ce; c0 += CH) {
        const int64_t c1 = (c0 + CH < ce) ? c0 + CH : ce;
        int64_t j = c0;
        for (; j + JB <= c1; j += JB)
            ksym_step<KIND, DM, NR, R, JB, OFFD, A32>(n, xa, sqn, c, u, j, c0, xi, mhn, ui, acc,
                                                      colw[wave], lane);
        for (; j < c1; ++j)
            ksym_step<KIND, DM, NR, R, 1, OFFD, A32>(n, xa, sqn, c, u, j, c0, xi, mhn, ui, acc,
                                                     colw[wave], lane);
        if (OFFD) {
            __syncthreads();
            const int64_t jj = c0 + threadIdx.x;
            if (threadIdx.x < CH && jj < c1) {
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const int e = threadIdx.x * NR + q;
                    const double v = (colw[0][e] + colw[1][e]) + (colw[2][e] + colw[3][e]);
                    part[(colslot * NR + q) * n + jj] = v;
                }
            }
            __syncthreads();
        }
    }
}

template <int KIND, int DM, int NR, bool A32>
__global__ __launch_bounds__(KS_THREADS) void k_ksym_f32(int64_t n, const float* __restrict__ xa,
                                                         const float* __restrict__ sqn, float c,
                                                         const double* __restrict__ u,
                                                         double* __restrict__ part, int nb, int S,
                                                         int CL, const int32_t* __restrict__ stop) {
    if (stop && *stop) return;
    constexpr int R = ksym_rows_ct(DM, NR, A32);
    constexpr int RB = KS_THREADS * R;
    __shared__ double colw[4][ks_chunk_ct(NR) * NR];

    // item -> (bi, bj, s): tiles enumerated row by row over the upper triangle
    int64_t t = blockIdx.x / S;
    const int s = (int)(blockIdx.x - t * S);
    int bi = 0;
    while (t >= nb - bi) { t -= nb - bi; ++bi; }
    const int bj = bi + (int)t;
    const int64_t row0 = (int64_t)bi * RB;
    const int64_t cb = (int64_t)bj * RB + (int64_t)s * CL;
    int64_t ce = cb + CL;
    if (ce > (int64_t)(bj + 1) * RB) ce = (int64_t)(bj + 1) * RB;
    if (ce > n) ce = n;

    float xi[R][DM];
    float mhn[R];
    typename KsymT<A32>::U ui[R][NR];
    double acc[R][NR];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = row0 + (int64_t)r * KS_THREADS + threadIdx.x;
        const int64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int k = 0; k < DM; ++k) xi[r][k] = xa[ic * DM + k];
        mhn[r] = -0.5f * sqn[ic];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            ui[r][q] = i < n ? (typename KsymT<A32>::U)u[(int64_t)q * n + i] : 0;
            acc[r][q] = 0.0;
        }
    }
    if (bj != bi)
        ksym_columns<KIND, DM, NR, true, A32>(n, xa, sqn, c, u, part, cb, ce, (int64_t)bi * S, xi,
                                             mhn, ui, acc, colw);
    else
        ksym_columns<KIND, DM, NR, false, A32>(n, xa, sqn, c, u, part, cb, ce, 0, xi, mhn, ui, acc,
                                              colw);
    const int64_t rslot = (int64_t)bj * S + s;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = row0 + (int64_t)r * KS_THREADS + threadIdx.x;
        if (i < n)
#pragma unroll
            for (int q = 0; q < NR; ++q) part[(rslot * NR + q) * n + i] = acc[r][q];
    }
}

// y_q = scale * (sum of the row's slots) + mu u_q, with partials of u_q^T y_q.
__global__ __launch_bounds__(256) void k_ksym_finish(int64_t n, int RB, int nb, int S, int nr,
                                                     const double* __restrict__ part, double scale,
                                                     double mu, const double* __restrict__ u,
                                                     double* __restrict__ y,
                                                     double* __restrict__ dot_part,
                                                     const int32_t* __restrict__ stop) {
    __shared__ double sc[4];
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int b = (int)(i / RB);
    for (int q = 0; q < nr; ++q) {
        double dot = 0.0;
        if (i < n) {
            // slots in a fixed order, four running sums so that loads stay in flight
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            int p = 0;
            for (; p + 4 <= b; p += 4)
#pragma unroll
                for (int u = 0; u < 4; ++u) s4[u] += part[((int64_t)(p + u) * S * nr + q) * n + i];
            for (; p < b; ++p) s4[0] += part[((int64_t)p * S * nr + q) * n + i];
            const int64_t z1 = (int64_t)nb * S;
            int64_t z = (int64_t)b * S;
            for (; z + 4 <= z1; z += 4)
#pragma unroll
                for (int u = 0; u < 4; ++u) s4[u] += part[((z + u) * nr + q) * n + i];
            for (; z < z1; ++z) s4[0] += part[(z * nr + q) * n + i];
            const double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            const double ui = u[(int64_t)q * n + i];
            const double yi = fma(scale, s, mu * ui);
            y[(int64_t)q * n + i] = yi;
            dot = ui * yi;
        }
        dot = block_sum(dot, sc);
        if (threadIdx.x == 0) dot_part[(int64_t)q * gridDim.x + blockIdx.x] = dot;
    }
}

template <int KIND, int NR, bool A32>
static void ksym_dispatch(const KernelOp& op, float c, const double* u, double* ws,
                          const KsymPlan& p, const int32_t* stop, hipStream_t st) {
    const unsigned grid = (unsigned)p.items;
#define KSL(DD) k_ksym_f32<KIND, DD, NR, A32><<<grid, KS_THREADS, 0, st>>>(op.n, op.xa, op.sqn, c, u, ws, p.nb, p.S, p.CL, stop)
    switch (op.dm) {
        case 4: KSL(4); break;
        case 8: KSL(8); break;
        case 16: KSL(16); break;
        default: KSL(32); break;
    }
#undef KSL
}

// Stage 1 + finish for nr in {1, 2, 4, 8} columns (u, y column-major with leading
// dimension n); a32 (nr <= 2 only) selects the float32 estimate-grade sums.
void launch_kernel_matvec_sym(const KernelOp& op, const double* u, int nr, double mu, double* y,
                              double* dot_part, double* ws, const int32_t* stop, hipStream_t st,
                              bool a32) {
    a32 = a32 && nr <= 2;
    const KsymPlan p = ksym_plan(op.n, op.d, nr, a32);
    const float c = kernel_c32(op.kind, op.kconst);
    {
        ProfScope prof(nr == 1 && !a32 ? PROF_KERNEL_MATVEC : -1, st);
#define KSD(K)                                                                   \
    if (a32) {                                                                   \
        if (nr == 1) ksym_dispatch<K, 1, true>(op, c, u, ws, p, stop, st);       \
        else ksym_dispatch<K, 2, true>(op, c, u, ws, p, stop, st);               \
    } else {                                                                     \
        switch (nr) {                                                            \
            case 1: ksym_dispatch<K, 1, false>(op, c, u, ws, p, stop, st); break; \
            case 2: ksym_dispatch<K, 2, false>(op, c, u, ws, p, stop, st); break; \
            case 4: ksym_dispatch<K, 4, false>(op, c, u, ws, p, stop, st); break; \
            default: ksym_dispatch<K, 8, false>(op, c, u, ws, p, stop, st); break; \
        }                                                                        \
    }
        if (op.kind == 1) { KSD(1) } else { KSD(2) }
#undef KSD
    }
    k_ksym_finish<<<(unsigned)((op.n + 255) / 256), 256, 0, st>>>(op.n, p.RB, p.nb, p.S, nr, ws,
                                                                  op.scale, mu, u, y, dot_part, stop);
}

// ===================================================================== float64
// The same pair-once scheme with float64 entries, for the float64 operator (the
// residual at restarts of the outer float64 refinement, certification, and the
// float64 working precision).  Points come as float64 records (coordinates, zero
// padding) and h_i = -g |x_i|^2 / 2; the thread's rows hold g x_i in registers and
// a column point streams through scalar loads, so an entry's exponent
//   t_ij = h_i + h_j + sum_k (g x_ik) x_jk = -g r_ij^2 / 2
// costs dm fused multiply-adds.  The RBF entry is 2^t; the Matern-3/2 entry
// (g = 1) is (1 + kconst r) 2^(-kconst r log2 e) with r = sqrt(-2 t).
//
// 2^t is the table-driven exp2_nonpos of kentry.hpp.

// Rows per thread and the work split do not depend on the number of columns, so a
// column goes through the same arithmetic alone and inside a two-column product.
constexpr int ks64_rows(int DM, int NR) { return (void)NR, DM <= 16 ? 4 : 2; }
constexpr int ks64_jb(int DM) { return DM <= 4 ? 4 : DM <= 8 ? 2 : 1; }
constexpr int KS64_CH = 256;

static KsymPlan ksym64_plan(int64_t n, int d, int nr) {
    KsymPlan p;
    p.R = ks64_rows(kernel_record_len(d), nr);
    p.RB = KS_THREADS * p.R;
    p.nb = (int)((n + p.RB - 1) / p.RB);
    const int64_t tiles = (int64_t)p.nb * (p.nb + 1) / 2;
    const int64_t target = 2048;
    int64_t S = (target + tiles - 1) / tiles;
    S = std::min<int64_t>(S, std::max(1, p.RB / 64));
    S = std::max<int64_t>(S, 1);
    p.S = (int)S;
    p.CL = (p.RB + p.S - 1) / p.S;
    p.items = tiles * p.S;
    return p;
}

size_t kernel_sym64_ws_doubles(int64_t n, int d, int nr) {
    const KsymPlan p = ksym64_plan(n, d, nr);
    return (size_t)p.nb * p.S * nr * (size_t)n;
}

template <int KIND, int DM, int NR, int R, int JB, bool OFFD>
RR_DEV void ks64_step(int64_t n, const double* __restrict__ xd, const double* __restrict__ hd, double kconst,
                      const double* __restrict__ u, int64_t j, int64_t c0, const double (&ai)[R][DM],
                      const double (&hi)[R], const double (&ui)[R][NR], double (&acc)[R][NR], double* colw,
                      int lane, const double* __restrict__ tab) {
    double cp[JB * NR];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
        const int64_t jj = j + jb;
        const double hj = hd[jj];
        double uj[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) uj[q] = u[(int64_t)q * n + jj];
        double t[R];
#pragma unroll
        for (int r = 0; r < R; ++r) t[r] = hi[r] + hj;
        const double* xj = xd + jj * DM;
#pragma unroll
        for (int k = 0; k < DM; ++k) {
            const double xjk = xj[k];
#pragma unroll
            for (int r = 0; r < R; ++r) t[r] = fma(ai[r][k], xjk, t[r]);
        }
        double kv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) kv[r] = kentry64<KIND>(t[r], kconst, tab);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[r][q] = fma(kv[r], uj[q], acc[r][q]);
        if (OFFD) {
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                double c = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) c = fma(kv[r], ui[r][q], c);
                cp[jb * NR + q] = c;
            }
        }
    }
    if (OFFD) {
        wave_sum_to63(cp);
        if (lane == 63) {
            const int base = (int)(j - c0) * NR;
#pragma unroll
            for (int m = 0; m < JB * NR; ++m) colw[base + m] = cp[m];
        }
    }
}

template <int KIND, int DM, int NR, bool OFFD>
RR_DEV void ks64_columns(int64_t n, const double* __restrict__ xd, const double* __restrict__ hd, double kconst,
                         const double* __restrict__ u, double* __restrict__ part, int64_t cb, int64_t ce,
                         int64_t colslot, const double (&ai)[ks64_rows(DM, NR)][DM], const double (&hi)[ks64_rows(DM, NR)],
                         const double (&ui)[ks64_rows(DM, NR)][NR], double (&acc)[ks64_rows(DM, NR)][NR],
                         double (*colw)[KS64_CH * NR], const double* __restrict__ tab) {
    constexpr int R = ks64_rows(DM, NR);
    constexpr int JB = ks64_jb(DM);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t c0 = cb; c0 < ce; c0 += KS64_CH) {
        const int64_t c1 = (c0 + KS64_CH < ce) ? c0 + KS64_CH : ce;
        int64_t j = c0;
        for (; j + JB <= c1; j += JB)
            ks64_step<KIND, DM, NR, R, JB, OFFD>(n, xd, hd, kconst, u, j, c0, ai, hi, ui, acc, colw[wave], lane,
                                                  tab);
        for (; j < c1; ++j)
            ks64_step<KIND, DM, NR, R, 1, OFFD>(n, xd, hd, kconst, u, j, c0, ai, hi, ui, acc, colw[wave], lane,
                                                 tab);
        if (OFFD) {
            __syncthreads();
            const int64_t jj = c0 + threadIdx.x;
            if (threadIdx.x < KS64_CH && jj < c1) {
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const int e = threadIdx.x * NR + q;
                    const double v = (colw[0][e] + colw[1][e]) + (colw[2][e] + colw[3][e]);
                    part[(colslot * NR + q) * n + jj] = v;
                }
            }
            __syncthreads();
        }
    }
}

template <int KIND, int DM, int NR>
__global__ __launch_bounds__(KS_THREADS) void k_ksym_f64(int64_t n, const double* __restrict__ xd,
                                                         const double* __restrict__ hd, double g,
                                                         double kconst, const double* __restrict__ u,
                                                         double* __restrict__ part, int nb, int S, int CL,
                                                         const int32_t* __restrict__ stop) {
    if (stop && *stop) return;
    constexpr int R = ks64_rows(DM, NR);
    constexpr int RB = KS_THREADS * R;
    __shared__ double colw[4][KS64_CH * NR];
    __shared__ double tab[EXP2_TAB];
    exp2_table_fill(tab);

    int64_t t = blockIdx.x / S;
    const int s = (int)(blockIdx.x - t * S);
    int bi = 0;
    while (t >= nb - bi) { t -= nb - bi; ++bi; }
    const int bj = bi + (int)t;
    const int64_t row0 = (int64_t)bi * RB;
    const int64_t cb = (int64_t)bj * RB + (int64_t)s * CL;
    int64_t ce = cb + CL;
    if (ce > (int64_t)(bj + 1) * RB) ce = (int64_t)(bj + 1) * RB;
    if (ce > n) ce = n;

    double ai[R][DM], hi[R], ui[R][NR], acc[R][NR];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = row0 + (int64_t)r * KS_THREADS + threadIdx.x;
        const int64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int k = 0; k < DM; ++k) ai[r][k] = g * xd[ic * DM + k];
        hi[r] = hd[ic];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            ui[r][q] = i < n ? u[(int64_t)q * n + i] : 0.0;
            acc[r][q] = 0.0;
        }
    }
    __syncthreads();   // the exp2 table
    if (bj != bi)
        ks64_columns<KIND, DM, NR, true>(n, xd, hd, kconst, u, part, cb, ce, (int64_t)bi * S, ai, hi, ui, acc,
                                         colw, tab);
    else
        ks64_columns<KIND, DM, NR, false>(n, xd, hd, kconst, u, part, cb, ce, 0, ai, hi, ui, acc, colw, tab);
    const int64_t rslot = (int64_t)bj * S + s;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = row0 + (int64_t)r * KS_THREADS + threadIdx.x;
        if (i < n)
#pragma unroll
            for (int q = 0; q < NR; ++q) part[(rslot * NR + q) * n + i] = acc[r][q];
    }
}

void launch_kernel_matvec_sym64(const KernelOp& op, const double* u, int nr, double mu, double* y,
                                double* dot_part, double* ws, const int32_t* stop, hipStream_t st) {
    const KsymPlan p = ksym64_plan(op.n, op.d, nr);
    const double g = kernel_g64(op.kind, op.kconst);
    const unsigned grid = (unsigned)p.items;
#define K64(K, DD, Q) k_ksym_f64<K, DD, Q><<<grid, KS_THREADS, 0, st>>>(op.n, op.xd, op.hd, g, op.kconst, u, ws, p.nb, p.S, p.CL, stop)
#define K64D(K, Q)                      \
    switch (op.dm) {                    \
        case 4: K64(K, 4, Q); break;    \
        case 8: K64(K, 8, Q); break;    \
        case 16: K64(K, 16, Q); break;  \
        default: K64(K, 32, Q); break;  \
    }
    {
        ProfScope prof(nr == 1 ? PROF_KERNEL_MATVEC64 : -1, st);
        if (op.kind == 1) {
            if (nr == 1) { K64D(1, 1) } else { K64D(1, 2) }
        } else {
            if (nr == 1) { K64D(2, 1) } else { K64D(2, 2) }
        }
    }
#undef K64D
#undef K64
    k_ksym_finish<<<(unsigned)((op.n + 255) / 256), 256, 0, st>>>(op.n, p.RB, p.nb, p.S, nr, ws, op.scale, mu,
                                                                  u, y, dot_part, stop);
}

}  // namespace rr
