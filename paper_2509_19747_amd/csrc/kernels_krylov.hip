// Kernels of the general Krylov engine (krylov.cpp): preconditioned MINRES with
// device-resident scalars (the MINRES branch of Algorithm RandRAND_PCG, and MINRES
// on the R-RandRAND operators of Algorithms RandRAND_CG / RandRAND_CG_split), plus
// the small pieces the R-RandRAND operator B u = (I-Pi) A_mu (I-Pi) u + tau Pi u
// needs.
//
// MINRES (Paige and Saunders 1975) with a preconditioner: preconditioned Lanczos
// (v_k = z_k / beta_k, z_k = P r_k, beta_k^2 = r_k^T z_k), Givens QR of the
// tridiagonal, and the three-term search-direction update
// w_k = (v_k - eps_k w_{k-2} - delta_k w_{k-1}) / gamma_k; the solution moves by
// phi_k w_k and its 2-norm residual by -phi_k (op w_k), where op w_k follows the
// same recurrence from op v_k.  One block of 1024 threads does the scalar steps.
#include "common.hpp"
#include "kernels.hpp"

#include <cfloat>

namespace rr {

constexpr int KV = 256;

static int kv_blocks(int64_t n) { return vec_blocks(n); }

// v = z / beta
__global__ __launch_bounds__(KV) void k_mr_v(int64_t n, const double* __restrict__ z, double* __restrict__ v,
                                             const MrState* s) {
    if (s->stop) return;
    const double ib = 1.0 / s->beta;
    for (int64_t i = (int64_t)blockIdx.x * KV + threadIdx.x; i < n; i += (int64_t)gridDim.x * KV)
        v[i] = z[i] * ib;
}

// t = av - (beta / oldb) r1 (no r1 term in a cycle's first step); partials of v^T t
__global__ __launch_bounds__(KV) void k_mr_t(int64_t n, const double* __restrict__ av,
                                             const double* __restrict__ r1, const double* __restrict__ v,
                                             double* __restrict__ t, const MrState* s, double* __restrict__ part) {
    __shared__ double sc[KV / WAVE];
    if (s->stop) return;
    const double f = s->k > 0 ? s->beta / s->oldb : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * KV + threadIdx.x; i < n; i += (int64_t)gridDim.x * KV) {
        const double ti = fma(-f, r1[i], av[i]);
        t[i] = ti;
        acc = fma(v[i], ti, acc);
    }
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void k_mr_alfa(const double* __restrict__ part, int count, MrState* s) {
    __shared__ double sc[16];
    if (s->stop) return;
    const double a = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) s->alfa = a;
}

// r1 <- r2, r2 <- t - (alfa / beta) r2
__global__ __launch_bounds__(KV) void k_mr_shift(int64_t n, const double* __restrict__ t, double* __restrict__ r1,
                                                 double* __restrict__ r2, const MrState* s) {
    if (s->stop) return;
    const double f = s->alfa / s->beta;
    for (int64_t i = (int64_t)blockIdx.x * KV + threadIdx.x; i < n; i += (int64_t)gridDim.x * KV) {
        const double r2i = r2[i];
        r1[i] = r2i;
        r2[i] = fma(-f, r2i, t[i]);
    }
}

// beta_{k+1} from the partials of r2^T z, then the rotations
__global__ void k_mr_rot(const double* __restrict__ part, int count, MrState* s) {
    __shared__ double sc[16];
    if (s->stop) return;
    const double b2 = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) {
        if (!(b2 >= 0.0) || !isfinite(b2)) {
            s->stop = STOP_BREAKDOWN;
            return;
        }
        const double beta = sqrt(b2);
        s->oldb = s->beta;
        s->beta = beta;
        const double oldeps = s->epsln;
        const double delta = s->cs * s->dbar + s->sn * s->alfa;
        const double gbar = s->sn * s->dbar - s->cs * s->alfa;
        s->epsln = s->sn * beta;
        s->dbar = -s->cs * beta;
        const double gamma = hypot(gbar, beta);
        if (!(gamma > 0.0)) {
            s->stop = STOP_BREAKDOWN;
            return;
        }
        s->cs = gbar / gamma;
        s->sn = beta / gamma;
        s->phi = s->cs * s->phibar;
        s->phibar = s->sn * s->phibar;
        s->gamma = gamma;
        s->delta = delta;
        s->oldeps = oldeps;
    }
}

// w2 <- w, w <- (v - oldeps w2_old - delta w) / gamma (same for aw from av);
// y += phi w; res -= phi aw; partials of ||res||^2
__global__ __launch_bounds__(KV) void k_mr_update(int64_t n, const double* __restrict__ v,
                                                  const double* __restrict__ av, double* __restrict__ w,
                                                  double* __restrict__ w2, double* __restrict__ aw,
                                                  double* __restrict__ aw2, double* __restrict__ y,
                                                  double* __restrict__ res, const MrState* s,
                                                  double* __restrict__ part) {
    __shared__ double sc[KV / WAVE];
    if (s->stop) return;
    const double ig = 1.0 / s->gamma, oe = s->oldeps, de = s->delta, phi = s->phi;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * KV + threadIdx.x; i < n; i += (int64_t)gridDim.x * KV) {
        const double w1 = w2[i], wo = w[i];
        const double wn = (v[i] - oe * w1 - de * wo) * ig;
        w2[i] = wo;
        w[i] = wn;
        const double a1 = aw2[i], ao = aw[i];
        const double an = (av[i] - oe * a1 - de * ao) * ig;
        aw2[i] = ao;
        aw[i] = an;
        y[i] = fma(phi, wn, y[i]);
        const double ri = fma(-phi, an, res[i]);
        res[i] = ri;
        acc = fma(ri, ri, acc);
    }
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// ||res||^2, iteration count, history, stop tests
__global__ void k_mr_rr(const double* __restrict__ part, int count, MrState* s) {
    __shared__ double sc[16];
    if (s->stop) return;
    const double rr = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) {
        s->rr = rr;
        const int it = s->iters + 1;
        s->iters = it;
        s->k += 1;
        if (s->hist && it < s->hist_cap) s->hist[it] = rr;
        if (!isfinite(rr)) s->stop = STOP_BREAKDOWN;
        else if (rr <= s->target2) s->stop = STOP_TARGET;
        else if (s->beta == 0.0) s->stop = STOP_TARGET;   // invariant Krylov space: solved in it
        else if (it >= s->maxit) s->stop = STOP_MAXIT;
    }
}

// cycle start: r1 = r2 = res = rhs was copied by the host code; z = P rhs with
// partials of rhs^T z in part
__global__ void k_mr_init(const double* __restrict__ part, int count, MrState* s, double target2, int32_t maxit,
                          int32_t iters, double* hist, int32_t hist_cap) {
    __shared__ double sc[16];
    const double b2 = block_sum_array(part, count, sc);
    if (threadIdx.x == 0) {
        s->beta = sqrt(fmax(b2, 0.0));
        s->oldb = 0.0;
        s->alfa = 0.0;
        s->dbar = 0.0;
        s->epsln = 0.0;
        s->phibar = s->beta;
        s->cs = -1.0;
        s->sn = 0.0;
        s->phi = s->gamma = s->delta = s->oldeps = 0.0;
        s->rr = 0.0;
        s->target2 = target2;
        s->iters = iters;
        s->maxit = maxit;
        s->k = 0;
        s->hist = hist;
        s->hist_cap = hist_cap;
        s->stop = (!(b2 > 0.0) || !isfinite(b2)) ? (b2 == 0.0 ? STOP_TARGET : STOP_BREAKDOWN) : STOP_NONE;
    }
}

void launch_mr_v(int64_t n, const double* z, double* v, const MrState* s, hipStream_t st) {
    k_mr_v<<<kv_blocks(n), KV, 0, st>>>(n, z, v, s);
}
void launch_mr_t(int64_t n, const double* av, const double* r1, const double* v, double* t, const MrState* s,
                 double* part, hipStream_t st) {
    k_mr_t<<<kv_blocks(n), KV, 0, st>>>(n, av, r1, v, t, s, part);
}
void launch_mr_alfa(const double* part, int count, MrState* s, hipStream_t st) {
    k_mr_alfa<<<1, 1024, 0, st>>>(part, count, s);
}
void launch_mr_shift(int64_t n, const double* t, double* r1, double* r2, const MrState* s, hipStream_t st) {
    k_mr_shift<<<kv_blocks(n), KV, 0, st>>>(n, t, r1, r2, s);
}
void launch_mr_rot(const double* part, int count, MrState* s, hipStream_t st) {
    k_mr_rot<<<1, 1024, 0, st>>>(part, count, s);
}
void launch_mr_update(int64_t n, const double* v, const double* av, double* w, double* w2, double* aw,
                      double* aw2, double* y, double* res, const MrState* s, double* part, hipStream_t st) {
    k_mr_update<<<kv_blocks(n), KV, 0, st>>>(n, v, av, w, w2, aw, aw2, y, res, s, part);
}
void launch_mr_rr(const double* part, int count, MrState* s, hipStream_t st) {
    k_mr_rr<<<1, 1024, 0, st>>>(part, count, s);
}
void launch_mr_init(const double* part, int count, MrState* s, double target2, int32_t maxit, int32_t iters,
                    double* hist, int32_t hist_cap, hipStream_t st) {
    k_mr_init<<<1, 1024, 0, st>>>(part, count, s, target2, maxit, iters, hist, hist_cap);
}

// dst = src with partials of ||src||^2 (the identity preconditioner's step)
__global__ __launch_bounds__(KV) void k_copy_dot(int64_t n, const double* __restrict__ src, double* __restrict__ dst,
                                                 double* __restrict__ part, const int32_t* __restrict__ stop) {
    __shared__ double sc[KV / WAVE];
    if (stop && *stop) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * KV + threadIdx.x; i < n; i += (int64_t)gridDim.x * KV) {
        const double x = src[i];
        dst[i] = x;
        acc = fma(x, x, acc);
    }
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
void launch_copy_dot(int64_t n, const double* src, double* dst, double* part, const int32_t* stop, hipStream_t st) {
    k_copy_dot<<<kv_blocks(n), KV, 0, st>>>(n, src, dst, part, stop);
}

// partials of a^T b, skipped once the stop word is set
__global__ __launch_bounds__(KV) void k_dot_part_stop(int64_t n, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ part,
                                                      const int32_t* __restrict__ stop) {
    __shared__ double sc[KV / WAVE];
    if (stop && *stop) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * KV + threadIdx.x; i < n; i += (int64_t)gridDim.x * KV)
        acc = fma(a[i], b[i], acc);
    acc = block_sum(acc, sc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
void launch_dot_part_stop(int64_t n, const double* a, const double* b, double* part, const int32_t* stop,
                          hipStream_t st) {
    k_dot_part_stop<<<kv_blocks(n), KV, 0, st>>>(n, a, b, part, stop);
}

// d = K1 c1 + K2 c2 for symmetric k x k K1, K2 and c1, c2 given as chunk partials
// (c_j = sum over chunks, added in chunk order); one thread per output row.
__global__ __launch_bounds__(256) void k_core_apply2(int64_t k, const double* __restrict__ K1,
                                                     const double* __restrict__ K2, int64_t ldk,
                                                     const double* __restrict__ c1p, const double* __restrict__ c2p,
                                                     int nchunks, double* __restrict__ d,
                                                     const int32_t* __restrict__ stop) {
    extern __shared__ double cs[];   // 2k: c1, c2
    if (stop && *stop) return;
    for (int64_t j = threadIdx.x; j < k; j += blockDim.x) {
        double a = 0.0, b = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) {
            a += c1p[(int64_t)ch * k + j];
            b += c2p[(int64_t)ch * k + j];
        }
        cs[j] = a;
        cs[k + j] = b;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    double s = 0.0;
    for (int64_t j = 0; j < k; ++j) {
        s = fma(K1[j + i * ldk], cs[j], s);
        s = fma(K2[j + i * ldk], cs[k + j], s);
    }
    d[i] = s;
}
void launch_core_apply2(int64_t k, const double* K1, const double* K2, int64_t ldk, const double* c1_part,
                        const double* c2_part, int nchunks, double* d, const int32_t* stop, hipStream_t st) {
    const int g = (int)((k + 255) / 256);
    k_core_apply2<<<g, 256, (size_t)2 * k * sizeof(double), st>>>(k, K1, K2, ldk, c1_part, c2_part, nchunks, d,
                                                                   stop);
}

}  // namespace rr
