// Kernel-block products for the basis-less C-RandRAND (Section 4.2, Algorithm
// BL_RandRAND_PCG) with a signed column-sampling test matrix: column c of Omega is
// sgn_c e_{idx_c}, so Y = A_mu Omega holds l columns of A_mu,
//   Y[i, c] = sgn_c (scale K(x_i, x_{idx_c}) + mu [i == idx_c]),
// and Q = Y R^{-1} is never stored: Q^T u = R^{-T} Y^T u and Q d = Y R^{-1} d cost one
// n x l block of kernel entries each instead of an n x l basis in memory.
//
// Entries: float32-class (the symmetric float32 formula of kentry.hpp from the
// float32 records, float64 sums) or float64 (the float64 records and the
// table-driven exp2 of the float64 symmetric matvec), by the handle's precision.
#include "common.hpp"
#include "kentry.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <type_traits>

namespace rr {

constexpr int KB_THREADS = 256;
constexpr double KB_LN2 = 0.69314718055994530942;
constexpr double KB_LOG2E = 1.44269504088896340736;

// 2^t for t <= 0, table-driven as in the float64 symmetric matvec (Tang's method).
RR_DEV double kb_exp2(double t, const double* __restrict__ tab) {
    t = fmax(t, -1100.0);
    const double kf = rint(t * 32.0);
    const double f = fma(kf, -0.03125, t);
    const int k = (int)kf;
    const double z = f * KB_LN2;
    double p = fma(z, 1.0 / 720.0, 1.0 / 120.0);
    p = fma(z, p, 1.0 / 24.0);
    p = fma(z, p, 1.0 / 6.0);
    p = fma(z, p, 0.5);
    p = fma(z, p, 1.0);
    p = fma(z, p, 1.0);
    return ldexp(tab[k & 31] * p, k >> 5);
}

// One kernel entry between points i and j (without scale).
template <int KIND, bool F64>
RR_DEV double kb_entry(const KernelOp& op, int64_t i, int64_t j, float c32, double g, const double* tab) {
    const int dm = op.dm;
    if constexpr (F64) {
        const double* xi = op.xd + i * dm;
        const double* xj = op.xd + j * dm;
        double t = op.hd[i] + op.hd[j];
        for (int k = 0; k < dm; ++k) t = fma(g * xi[k], xj[k], t);
        if (KIND == 1) return kb_exp2(t, tab);
        const double kr = op.kconst * sqrt(fmax(-2.0 * t, 0.0));
        return (1.0 + kr) * kb_exp2(-kr * KB_LOG2E, tab);
    } else {
        const float* xi = op.xa + i * dm;
        const float* xj = op.xa + j * dm;
        float s = kpair_init(-0.5f * op.sqn[i], op.sqn[j]);
        for (int k = 0; k < dm; ++k) s = fmaf(xi[k], xj[k], s);
        return (double)kval32<KIND>(s, c32);
    }
}

RR_DEV void kb_table(double* tab) {
    if (threadIdx.x < 32) tab[threadIdx.x] = exp2((double)threadIdx.x / 32.0);
    __syncthreads();
}

// The records of a kernel entry held by one side: the float32 path keeps x and
// -|x|^2 / 2, the float64 path g x and h = -g |x|^2 / 2 (the operands kb_entry uses).
// An entry between a held side a (the "i" of kb_entry) and a streamed side b is
// computed in kb_entry's order, so both forms give the same value.
template <bool F64, int DM>
struct KbSide {
    using T = std::conditional_t<F64, double, float>;
    T x[DM];
    T h;   // F32: -0.5 |x|^2 (the i side) or |x|^2 (the j side); F64: h
};
template <bool F64, int DM>
RR_DEV void kb_load(const KernelOp& op, int64_t i, double g, bool as_i, KbSide<F64, DM>& o) {
    if constexpr (F64) {
        const double* xi = op.xd + i * DM;
#pragma unroll
        for (int k = 0; k < DM; ++k) o.x[k] = as_i ? g * xi[k] : xi[k];
        o.h = op.hd[i];
    } else {
        const float* xi = op.xa + i * DM;
#pragma unroll
        for (int k = 0; k < DM; ++k) o.x[k] = xi[k];
        o.h = as_i ? -0.5f * op.sqn[i] : op.sqn[i];
    }
}
// entry (without scale) between i-side a and j-side b (kb_entry<KIND, F64>(op, i, j))
template <int KIND, bool F64, int DM, typename A, typename B>
RR_DEV double kb_entry_r(const A& ax, double ah, const B& bx, double bh, float c32, double kconst,
                         const double* tab) {
    if constexpr (F64) {
        double t = ah + bh;
#pragma unroll
        for (int k = 0; k < DM; ++k) t = fma((double)ax[k], (double)bx[k], t);
        if (KIND == 1) return kb_exp2(t, tab);
        const double kr = kconst * sqrt(fmax(-2.0 * t, 0.0));
        return (1.0 + kr) * kb_exp2(-kr * KB_LOG2E, tab);
    } else {
        float s = kpair_init((float)ah, (float)bh);
#pragma unroll
        for (int k = 0; k < DM; ++k) s = fmaf((float)ax[k], (float)bx[k], s);
        return (double)kval32<KIND>(s, c32);
    }
}

// out[c] = sgn_c (scale sum_j K(x_{idx_c}, x_j) v_j + mu v_{idx_c}).  Block: KB_RB
// sampled rows (their records in LDS, read as broadcasts) against every point j,
// one point per thread and pass, so a point's record is loaded once per KB_RB
// entries; the per-thread sums are added by a block reduction in a fixed order.
constexpr int KB_RB = 4;
template <int KIND, bool F64, int DM>
__global__ __launch_bounds__(KB_THREADS) void k_kblock_rows(KernelOp op, const int32_t* __restrict__ idx,
                                                            const double* __restrict__ sgn, int64_t l, float c32,
                                                            double g, const double* __restrict__ v, double mu,
                                                            double* __restrict__ out,
                                                            const int32_t* __restrict__ stop) {
    using T = typename KbSide<F64, DM>::T;
    __shared__ double tab[32];
    __shared__ double sc[KB_THREADS / WAVE];
    __shared__ T rx[KB_RB][DM];
    __shared__ T rh[KB_RB];
    if (stop && *stop) return;
    kb_table(tab);
    const int64_t c0 = (int64_t)blockIdx.x * KB_RB;
    if (threadIdx.x < KB_RB) {
        const int64_t c = c0 + threadIdx.x < l ? c0 + threadIdx.x : l - 1;
        KbSide<F64, DM> a;
        kb_load<F64, DM>(op, idx[c], g, true, a);
#pragma unroll
        for (int k = 0; k < DM; ++k) rx[threadIdx.x][k] = a.x[k];
        rh[threadIdx.x] = a.h;
    }
    __syncthreads();
    double acc[KB_RB];
#pragma unroll
    for (int r = 0; r < KB_RB; ++r) acc[r] = 0.0;
    for (int64_t j = threadIdx.x; j < op.n; j += KB_THREADS) {
        KbSide<F64, DM> b;
        kb_load<F64, DM>(op, j, g, false, b);
        const double vj = v[j];
#pragma unroll
        for (int r = 0; r < KB_RB; ++r)
            acc[r] = fma(kb_entry_r<KIND, F64, DM>(rx[r], (double)rh[r], b.x, (double)b.h, c32, op.kconst, tab), vj,
                         acc[r]);
    }
#pragma unroll
    for (int r = 0; r < KB_RB; ++r) {
        const double tot = block_sum(acc[r], sc);
        const int64_t c = c0 + r;
        if (threadIdx.x == 0 && c < l) {
            const int64_t ic = idx[c];
            out[c] = sgn[c] * fma(op.scale, tot, mu * v[ic]);
        }
    }
}

// z_i = rcoef r_i + scale sum_c K(x_i, x_{idx_c}) sgn_c d_c + mu sgn_{pos_i} d_{pos_i},
// with block partials of r^T z (rz_part may be null): thread per row (its record in
// registers), the sampled columns' records and sgn d staged in LDS in chunks and
// read as broadcasts.
constexpr int KB_CHUNK = 128;
template <int KIND, bool F64, int DM>
__global__ __launch_bounds__(KB_THREADS) void k_kblock_cols(KernelOp op, const int32_t* __restrict__ idx,
                                                            const double* __restrict__ sgn,
                                                            const int32_t* __restrict__ pos, int64_t l, float c32,
                                                            double g, const double* __restrict__ d, double mu,
                                                            const double* __restrict__ r, double rcoef,
                                                            double* __restrict__ z, double* __restrict__ rz_part,
                                                            const int32_t* __restrict__ stop) {
    using T = typename KbSide<F64, DM>::T;
    __shared__ double tab[32];
    __shared__ T cx[KB_CHUNK][DM];
    __shared__ T ch[KB_CHUNK];
    __shared__ double sd[KB_CHUNK];
    __shared__ double sc[KB_THREADS / WAVE];
    if (stop && *stop) return;
    kb_table(tab);
    const int64_t i = (int64_t)blockIdx.x * KB_THREADS + threadIdx.x;
    const int64_t ic = i < op.n ? i : op.n - 1;
    KbSide<F64, DM> a;
    kb_load<F64, DM>(op, ic, g, true, a);
    double acc = 0.0;
    for (int64_t c0 = 0; c0 < l; c0 += KB_CHUNK) {
        const int cn = (int)std::min<int64_t>(KB_CHUNK, l - c0);
        __syncthreads();
        for (int q = threadIdx.x; q < cn; q += KB_THREADS) {
            KbSide<F64, DM> b;
            kb_load<F64, DM>(op, idx[c0 + q], g, false, b);
#pragma unroll
            for (int k = 0; k < DM; ++k) cx[q][k] = b.x[k];
            ch[q] = b.h;
            sd[q] = sgn[c0 + q] * d[c0 + q];
        }
        __syncthreads();
        for (int q = 0; q < cn; ++q)
            acc = fma(kb_entry_r<KIND, F64, DM>(a.x, (double)a.h, cx[q], (double)ch[q], c32, op.kconst, tab), sd[q],
                      acc);
    }
    double dot = 0.0;
    if (i < op.n) {
        double zi = fma(op.scale, acc, r ? rcoef * r[i] : 0.0);
        const int32_t p = pos[i];
        if (p >= 0) zi = fma(mu * sgn[p], d[p], zi);
        z[i] = zi;
        if (r) dot = r[i] * zi;
    }
    if (rz_part) {
        dot = block_sum(dot, sc);
        if (threadIdx.x == 0) rz_part[blockIdx.x] = dot;
    }
}

// Rows of Y (row-major, out[i * ldo + c]): rows r0 + i (i < rows), or the sampled
// rows rowidx[i] scaled by rowsgn[i] (then the block is Omega^T Y).
template <int KIND, bool F64>
__global__ __launch_bounds__(KB_THREADS) void k_kblock_y(KernelOp op, const int32_t* __restrict__ idx,
                                                         const double* __restrict__ sgn, int64_t l, float c32,
                                                         double g, double mu, int64_t r0, int64_t rows,
                                                         const int32_t* __restrict__ rowidx,
                                                         const double* __restrict__ rowsgn,
                                                         double* __restrict__ out, int64_t ldo) {
    __shared__ double tab[32];
    kb_table(tab);
    const int64_t total = rows * l;
    for (int64_t e = (int64_t)blockIdx.x * KB_THREADS + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * KB_THREADS) {
        const int64_t i = e / l, c = e - i * l;
        const int64_t gi = rowidx ? (int64_t)rowidx[i] : r0 + i;
        const int64_t jc = idx[c];
        double y = op.scale * kb_entry<KIND, F64>(op, gi, jc, c32, g, tab);
        if (gi == jc) y += mu;
        y *= sgn[c];
        if (rowsgn) y *= rowsgn[i];
        out[i * ldo + c] = y;
    }
}

__global__ void k_colsample_prep(int64_t n, int64_t l, const float* __restrict__ D, const int32_t* __restrict__ idx,
                                 double* __restrict__ sgn, int32_t* __restrict__ pos) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pos[i] = -1;
    __syncthreads();   // single block: every pos is cleared before the scatter
    for (int64_t c = threadIdx.x; c < l; c += blockDim.x) {
        sgn[c] = (double)D[idx[c]];
        pos[idx[c]] = (int32_t)c;
    }
}

template <typename T>
__global__ void k_colsample_fill(int64_t n, int64_t l, int64_t ld, const int32_t* __restrict__ idx,
                                 const double* __restrict__ sgn, T* __restrict__ out) {
    const int64_t total = ld * l;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % ld, c = e / ld;
        out[e] = from_f64<T>(i == idx[c] ? sgn[c] : 0.0);
    }
}

// --------------------------------------------------------------- launchers
struct KbArgs {
    float c32;
    double g;
};
static KbArgs kb_args(const KernelOp& op) { return KbArgs{kernel_c32(op.kind, op.kconst), kernel_g64(op.kind, op.kconst)}; }

// f(integral_constant K, bool F64, int DM): the kernel template of this operator
template <typename F>
static void kb_dispatch(const KernelOp& op, bool f64, F&& f) {
    auto dm = [&](auto kk, auto ff) {
        switch (op.dm) {
            case 4: f(kk, ff, std::integral_constant<int, 4>{}); break;
            case 8: f(kk, ff, std::integral_constant<int, 8>{}); break;
            case 16: f(kk, ff, std::integral_constant<int, 16>{}); break;
            default: f(kk, ff, std::integral_constant<int, 32>{}); break;
        }
    };
    auto fl = [&](auto kk) {
        if (f64) dm(kk, std::true_type{});
        else dm(kk, std::false_type{});
    };
    if (op.kind == 1) fl(std::integral_constant<int, 1>{});
    else fl(std::integral_constant<int, 2>{});
}

void launch_kblock_rows(const KernelOp& op, bool f64, const int32_t* idx, const double* sgn, int64_t l,
                        const double* v, double mu, double* out, const int32_t* stop, hipStream_t st) {
    const KbArgs a = kb_args(op);
    const unsigned grid = (unsigned)((l + KB_RB - 1) / KB_RB);
    kb_dispatch(op, f64, [&](auto kk, auto ff, auto dd) {
        k_kblock_rows<decltype(kk)::value, decltype(ff)::value, decltype(dd)::value>
            <<<grid, KB_THREADS, 0, st>>>(op, idx, sgn, l, a.c32, a.g, v, mu, out, stop);
    });
}

int kblock_cols_blocks(int64_t n) { return (int)((n + KB_THREADS - 1) / KB_THREADS); }

void launch_kblock_cols(const KernelOp& op, bool f64, const int32_t* idx, const double* sgn, const int32_t* pos,
                        int64_t l, const double* d, double mu, const double* r, double rcoef, double* z,
                        double* rz_part, const int32_t* stop, hipStream_t st) {
    const KbArgs a = kb_args(op);
    const unsigned grid = (unsigned)kblock_cols_blocks(op.n);
    kb_dispatch(op, f64, [&](auto kk, auto ff, auto dd) {
        k_kblock_cols<decltype(kk)::value, decltype(ff)::value, decltype(dd)::value>
            <<<grid, KB_THREADS, 0, st>>>(op, idx, sgn, pos, l, a.c32, a.g, d, mu, r, rcoef, z, rz_part, stop);
    });
}

void launch_kblock_y(const KernelOp& op, bool f64, const int32_t* idx, const double* sgn, int64_t l, double mu,
                     int64_t r0, int64_t rows, const int32_t* rowidx, const double* rowsgn, double* out,
                     int64_t ldo, hipStream_t st) {
    const KbArgs a = kb_args(op);
    int64_t grid = (rows * l + KB_THREADS - 1) / KB_THREADS;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
#define KBY(K, F) k_kblock_y<K, F><<<(unsigned)grid, KB_THREADS, 0, st>>>(op, idx, sgn, l, a.c32, a.g, mu, r0, rows, rowidx, rowsgn, out, ldo)
    if (op.kind == 1) { if (f64) KBY(1, true); else KBY(1, false); }
    else { if (f64) KBY(2, true); else KBY(2, false); }
#undef KBY
}

void launch_colsample_prep(int64_t n, int64_t l, const float* D, const int32_t* idx, double* sgn, int32_t* pos,
                           hipStream_t st) {
    k_colsample_prep<<<1, 1024, 0, st>>>(n, l, D, idx, sgn, pos);
}

void launch_colsample_fill(int dtype, int64_t n, int64_t l, int64_t ld, const int32_t* idx, const double* sgn,
                           void* out, hipStream_t st) {
    int64_t g = (ld * l + 255) / 256;
    if (g > 65536) g = 65536;
    if (dtype == DT_F64) k_colsample_fill<double><<<(unsigned)g, 256, 0, st>>>(n, l, ld, idx, sgn, (double*)out);
    else if (dtype == DT_F32) k_colsample_fill<float><<<(unsigned)g, 256, 0, st>>>(n, l, ld, idx, sgn, (float*)out);
    else k_colsample_fill<__hip_bfloat16><<<(unsigned)g, 256, 0, st>>>(n, l, ld, idx, sgn, (__hip_bfloat16*)out);
}

}  // namespace rr
