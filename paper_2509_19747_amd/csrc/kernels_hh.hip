// Blocked Householder QR for the small tall matrices of the build: the sketch
// Theta Y (2k x k) whose R factor Algorithm prec_chol_qr needs, and the
// per-shift 2l x l reduced QR of the joint basis (Section 5.1), which also
// needs the explicit Q.
//
// Panels of NB = 16 (8 for more than 1024 rows) columns.  One 512-thread block
// factors a panel with the panel
// held in registers (thread t owns rows j0 + t + 512 r), producing the
// reflectors V, their scalars tau and the compact-WY factor T of the panel
// (Q_panel = H_1 ... H_NB = I - V T V^T), and the R entries of its columns.
// One more launch per panel updates the trailing columns with the three block
// products fused (k_hb_update),
//   W = V^T S_t,  W <- T^T W,  S_t <- S_t - V W,
// and an explicit Q is accumulated backwards panel by panel with
//   W = V^T Q_t,  W <- T W,  Q_t <- Q_t - V W.
// Each reflector is H = I - f v v^T with v_0 = alpha - beta, beta = -sign(alpha)
// ||x|| and f = 2 / v^T v (Golub and Van Loan, Algorithm 5.1.1, unnormalised).
// R's diagonal is made positive at the end (R <- D R, Q <- Q D with D = sign).
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <utility>

namespace rr {

constexpr int HB_THREADS = 512;
constexpr int HB_WAVES = HB_THREADS / WAVE;

// Block-wide sum of NV values per thread; every thread gets the totals (DPP
// tree within each wave, then the waves in a fixed order).
template <int NV>
RR_DEV void hb_block_sum(double (&v)[NV], double* red, double* tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    wave_sum_to63(v);
    if (lane == 63)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[w * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int i = 0; i < HB_WAVES; ++i) s += red[i * NV + threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = tot[q];
    __syncthreads();
}

// Block-wide sums of NV values per thread through LDS: every thread stores its NV
// partials, then the P = 512 / NV threads that share value q add 512 / P of them each
// and finish with a P-lane butterfly.  Far fewer instructions than NV wave-wide DPP
// trees for the panel's NB dot products.  Fixed order, so deterministic.
template <int NV>
RR_DEV void hb_block_sum_t(double (&v)[NV], double* buf, double* tot) {
    constexpr int P = HB_THREADS / NV;
    static_assert(P == 16 || P == 32 || P == 64, "NV must be 8, 16 or 32");
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) buf[q * HB_THREADS + t] = v[q];
    __syncthreads();
    const int q = t / P, part = t % P;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < HB_THREADS / P; ++j) s += buf[q * HB_THREADS + part + P * j];
#pragma unroll
    for (int o = P / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, P);
    if (part == 0) tot[q] = s;
    __syncthreads();
#pragma unroll
    for (int q2 = 0; q2 < NV; ++q2) v[q2] = tot[q2];
}

// f(integral_constant<int, C>) for C in the sequence, in order
template <typename F, int... C>
RR_DEV void hb_unrolled(F& f, std::integer_sequence<int, C...>) {
    (f(std::integral_constant<int, C>{}), ...);
}

// Factor columns [j0, j0 + nbe) of S (rows [j0, m)), nbe <= NB; m - j0 <= RR * 512.
// Writes V[:, j0..] (zeros above the diagonal), tau[j0..], T (NB x NB, column-major,
// ldt NB) and R[0:k, j0..] (rows above the panel from S, which already holds them).
template <int RR, int NB>
__global__ __launch_bounds__(HB_THREADS) void k_panel_qr(const double* __restrict__ S, int64_t m,
                                                         int64_t k, int64_t lds, int64_t j0, int nbe,
                                                         double* __restrict__ V, int64_t ldv,
                                                         double* __restrict__ tauv,
                                                         double* __restrict__ T,
                                                         double* __restrict__ R, int64_t ldr) {
    __shared__ double tot[NB];
    __shared__ double dbuf[NB * HB_THREADS];
    __shared__ double Tsh[NB * NB];
    __shared__ double prow[2][NB];
    const int t = threadIdx.x;
    double a[RR][NB];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
#pragma unroll
        for (int c = 0; c < NB; ++c) a[r][c] = (i < m && c < nbe) ? S[i + (j0 + c) * lds] : 0.0;
    }
    for (int i = t; i < NB * NB; i += HB_THREADS) Tsh[i] = 0.0;
    // R rows above the panel are final in S
    for (int c = 0; c < nbe; ++c)
        for (int64_t i = t; i < j0; i += HB_THREADS) R[i + (j0 + c) * ldr] = S[i + (j0 + c) * lds];
    __syncthreads();

    double rsave[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) rsave[c] = 0.0;
    // One block reduction per column.  With x = column c at rows >= kc and the
    // pivot-row entries p_q = a[kc][q], the sums s_q = x^T a_q (all panel columns,
    // q = c included) give everything the step needs:
    //   ||x||^2 = s_c,  v = x - beta e_kc,  v^T a_q = s_q - beta p_q,
    //   v^T v = v0^2 + (s_c - alpha^2)  (v0^2 >= alpha^2 dominates, so the
    //   difference costs no relative accuracy).
    // The previous reflectors (q < c) give V(:, q)^T v for T the same way.  The
    // pivot row is published through LDS, double-buffered so that a thread still
    // reading the previous column's entries never sees the next one's.
    // one instance per column, so that every register index is static
    auto column = [&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (c >= nbe) return;   // uniform over the block
        const int64_t kc = j0 + c;
        double* pr = prow[c & 1];
        // the pivot row kc is thread c, register row 0
        if (t == c)
#pragma unroll
            for (int q = 0; q < NB; ++q) pr[q] = a[0][q];
        double dots[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) dots[q] = 0.0;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
            const double x = (i >= kc && i < m) ? a[r][c] : 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q) dots[q] = fma(x, a[r][q], dots[q]);
        }
        hb_block_sum_t<NB>(dots, dbuf, tot);   // its barriers also publish the pivot row
        const double alpha = pr[c];
        const double sc = dots[c];
        const double normx = sqrt(sc);
        const double beta = (alpha >= 0.0) ? -normx : normx;
        const double v0 = alpha - beta;
        const double vtv = fma(v0, v0, sc - alpha * alpha);
        const double f = (vtv > 0.0) ? 2.0 / vtv : 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) dots[q] = fma(-beta, pr[q], dots[q]);
        // R entries of column kc in the panel rows (thread t < c holds row j0 + t, thread
        // c the diagonal) are kept in registers and stored after the loop: a global
        // store here would make every following barrier wait for it.
        if (t < c) rsave[c] = a[0][c];
        else if (t == c) rsave[c] = (normx > 0.0) ? beta : alpha;
        // v into column c (zeros above the pivot), then the columns still to be reduced
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
            const double v = (i < kc || i >= m) ? 0.0 : (i == kc ? v0 : a[r][c]);
            a[r][c] = v;
#pragma unroll
            for (int q = c + 1; q < NB; ++q)   // columns past nbe hold zeros and stay zero
                a[r][q] = fma(-f * dots[q], v, a[r][q]);
        }
        // T(:, c): T(c, c) = f, T(0:c, c) = -f T(0:c, 0:c) (V(:, 0:c)^T v); thread i
        // forms row i of T and reads only its own row, so no barrier is needed
        if (t < c) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j >= t && j < c) s = fma(Tsh[t + j * NB], dots[j], s);
            Tsh[t + c * NB] = -f * s;
        } else if (t == c) {
            Tsh[c + c * NB] = f;
        }
    };
    hb_unrolled(column, std::make_integer_sequence<int, NB>{});
    __syncthreads();
    // reflectors out (rows < j0 are zero)
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
        if (i < m)
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < nbe) V[i + (j0 + c) * ldv] = a[r][c];
    }
    for (int c = 0; c < nbe; ++c)
        for (int64_t i = t; i < j0; i += HB_THREADS) V[i + (j0 + c) * ldv] = 0.0;
    for (int i = t; i < NB * NB; i += HB_THREADS) T[i] = Tsh[i];
    if (t < nbe) tauv[j0 + t] = Tsh[t + t * NB];
    // R columns of the panel: rows [j0, j0 + c] from the registers, zeros below to row k
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c >= nbe) continue;
        if (t <= c) R[j0 + t + (j0 + c) * ldr] = rsave[c];
        for (int64_t i = j0 + c + 1 + t; i < k; i += HB_THREADS) R[i + (j0 + c) * ldr] = 0.0;
    }
}

// Trailing update after one panel, the three block products in one launch:
//   W = V_p^T X_t,  W <- T^T W (factoring) or T W (accumulating Q backwards),
//   X_t <- X_t - V_p W.
// Block b updates columns [c0 + CW b, c0 + CW b + CW) of X; thread t owns rows
// j0 + t + 512 r as in the panel kernel, so the NB x CW inner products are one
// block sum.  T is the panel's upper triangular compact-WY factor (NB x NB, ld NB).
template <int RR, int NB, int CW, bool TT>
__global__ __launch_bounds__(HB_THREADS) void k_hb_update(const double* __restrict__ V, int64_t ldv,
                                                          const double* __restrict__ T, int64_t m,
                                                          int64_t j0, int nbe, double* __restrict__ X,
                                                          int64_t ldx, int64_t c0, int64_t ncols) {
    __shared__ double red[HB_WAVES * NB * CW];
    __shared__ double tot[NB * CW];
    __shared__ double Tsh[NB * NB];
    __shared__ double w2s[NB * CW];
    const int t = threadIdx.x;
    for (int i = t; i < NB * NB; i += HB_THREADS) Tsh[i] = T[i];
    const int64_t cb = c0 + (int64_t)blockIdx.x * CW;
    double v[RR][NB], x[RR][CW];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
#pragma unroll
        for (int q = 0; q < NB; ++q) v[r][q] = (i < m && q < nbe) ? V[i + (j0 + q) * ldv] : 0.0;
#pragma unroll
        for (int j = 0; j < CW; ++j) x[r][j] = (i < m && cb + j < c0 + ncols) ? X[i + (cb + j) * ldx] : 0.0;
    }
    double w[NB * CW];
#pragma unroll
    for (int e = 0; e < NB * CW; ++e) w[e] = 0.0;
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int j = 0; j < CW; ++j) w[q * CW + j] = fma(v[r][q], x[r][j], w[q * CW + j]);
    hb_block_sum<NB * CW>(w, red, tot);   // its barriers also publish Tsh
    // op(T) W, one entry per thread: T^T W reads rows p <= q, T W rows p >= q
    if (t < NB * CW) {
        const int q = t / CW, j = t % CW;
        double s = 0.0;
        for (int p = 0; p < NB; ++p) {
            if (TT && p <= q) s = fma(Tsh[p + q * NB], tot[p * CW + j], s);
            if (!TT && p >= q) s = fma(Tsh[q + p * NB], tot[p * CW + j], s);
        }
        w2s[t] = s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            double y = x[r][j];
#pragma unroll
            for (int q = 0; q < NB; ++q) y = fma(-v[r][q], w2s[q * CW + j], y);
            if (i < m && cb + j < c0 + ncols) X[i + (cb + j) * ldx] = y;
        }
    }
}

// R <- D R and Q <- Q D with D = sign(diag(R)): strict upper part of R and Q
// first (they read the unchanged diagonal), then the diagonal.
__global__ void k_hb_sign_fix(double* R, int64_t k, int64_t ldr, double* Q, int64_t m, int64_t ldq) {
    const int64_t nq = Q ? m * k : 0;
    const int64_t total = nq + k * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < nq) {
            const int64_t j = e / m, i = e - j * m;
            if (R[j + j * ldr] < 0.0) Q[i + j * ldq] = -Q[i + j * ldq];
        } else {
            const int64_t e2 = e - nq;
            const int64_t j = e2 / k, i = e2 - j * k;   // R(i, j)
            if (i < j && R[i + i * ldr] < 0.0) R[i + j * ldr] = -R[i + j * ldr];
        }
    }
}
__global__ void k_hb_sign_fix_diag(double* R, int64_t k, int64_t ldr) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < k;
         j += (int64_t)gridDim.x * blockDim.x)
        if (R[j + j * ldr] < 0.0) R[j + j * ldr] = -R[j + j * ldr];
}
__global__ void k_hb_eye(double* Q, int64_t m, int64_t k, int64_t ldq) {
    const int64_t total = m * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / m, i = e - j * m;
        Q[i + j * ldq] = (i == j) ? 1.0 : 0.0;
    }
}

static int hb_grid(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 8192);
}

constexpr int HB_NB = 16;   // largest panel width

size_t householder_ws_doubles(int64_t m, int64_t k) {
    const int64_t panels = (k + HB_NB - 1) / HB_NB;
    return (size_t)m * k + k + (size_t)panels * HB_NB * HB_NB + 64;   // V, tau, the T factors
}

bool householder_blocked_ok(int64_t m, int64_t k) { return m <= 4 * HB_THREADS && k >= 1 && m >= k; }

template <int RR, int NB>
static void hb_panel(double* S, int64_t m, int64_t k, int64_t lds, int64_t j0, int nbe, double* V,
                     double* tauv, double* T, double* R, int64_t ldr, hipStream_t st) {
    k_panel_qr<RR, NB><<<1, HB_THREADS, 0, st>>>(S, m, k, lds, j0, nbe, V, m, tauv, T, R, ldr);
}

constexpr int HB_CW = 2;   // trailing columns per update block

// X[:, c0:c0+ncols] <- (I - V_p op(T) V_p^T) X[...] over rows [j0, m); op(T) = T^T
// when factoring (TT), T when accumulating Q.
template <int NB, bool TT>
static void hb_update(const double* V, int64_t m, const double* T, int64_t j0, int nbe, double* X,
                      int64_t ldx, int64_t c0, int64_t ncols, hipStream_t st) {
    const int64_t L = m - j0;
    const unsigned g = (unsigned)((ncols + HB_CW - 1) / HB_CW);
    if (L <= HB_THREADS)
        k_hb_update<1, NB, HB_CW, TT><<<g, HB_THREADS, 0, st>>>(V, m, T, m, j0, nbe, X, ldx, c0, ncols);
    else if (L <= 2 * HB_THREADS)
        k_hb_update<2, NB, HB_CW, TT><<<g, HB_THREADS, 0, st>>>(V, m, T, m, j0, nbe, X, ldx, c0, ncols);
    else if constexpr (NB == 8)
        k_hb_update<4, NB, HB_CW, TT><<<g, HB_THREADS, 0, st>>>(V, m, T, m, j0, nbe, X, ldx, c0, ncols);
}

// Shared driver: factor S panel by panel, update the trailing columns; when Q is
// given, accumulate it afterwards.  Panels of 16 columns while the panel rows
// fit 2 registers per thread, 8 columns beyond (4 rows per thread).
// ws: householder_ws_doubles(m, k).
static void hb_factor(double* S, int64_t m, int64_t k, int64_t lds, double* R, int64_t ldr,
                      double* Q, int64_t ldq, double* ws, size_t wsd, hipStream_t st) {
    (void)wsd;
    const int nb = m <= 2 * HB_THREADS ? 16 : 8;
    double* V = ws;
    double* tauv = V + (size_t)m * k;
    double* Tall = tauv + k;
    const int64_t panels = (k + nb - 1) / nb;
    for (int64_t p = 0; p < panels; ++p) {
        const int64_t j0 = p * nb;
        const int nbe = (int)std::min<int64_t>(nb, k - j0);
        double* T = Tall + (size_t)p * nb * nb;
        const int64_t L = m - j0;
        if (L <= HB_THREADS) {
            if (nb == 16) hb_panel<1, 16>(S, m, k, lds, j0, nbe, V, tauv, T, R, ldr, st);
            else hb_panel<1, 8>(S, m, k, lds, j0, nbe, V, tauv, T, R, ldr, st);
        } else if (L <= 2 * HB_THREADS) {
            if (nb == 16) hb_panel<2, 16>(S, m, k, lds, j0, nbe, V, tauv, T, R, ldr, st);
            else hb_panel<2, 8>(S, m, k, lds, j0, nbe, V, tauv, T, R, ldr, st);
        } else {
            hb_panel<4, 8>(S, m, k, lds, j0, nbe, V, tauv, T, R, ldr, st);
        }
        const int64_t jt = j0 + nbe, nt = k - jt;
        if (nt > 0) {
            if (nb == 16) hb_update<16, true>(V, m, T, j0, nbe, S, lds, jt, nt, st);
            else hb_update<8, true>(V, m, T, j0, nbe, S, lds, jt, nt, st);
        }
    }
    if (Q) {
        // Q = [I; 0], then Q_t <- Q_t - V_p (T (V_p^T Q_t)) for panels in reverse
        k_hb_eye<<<hb_grid(m * k), 256, 0, st>>>(Q, m, k, ldq);
        for (int64_t p = panels - 1; p >= 0; --p) {
            const int64_t j0 = p * nb;
            const int nbe = (int)std::min<int64_t>(nb, k - j0);
            const double* T = Tall + (size_t)p * nb * nb;
            if (nb == 16) hb_update<16, false>(V, m, T, j0, nbe, Q, ldq, j0, k - j0, st);
            else hb_update<8, false>(V, m, T, j0, nbe, Q, ldq, j0, k - j0, st);
        }
    }
    const int64_t tot = (Q ? m * k : 0) + k * k;
    k_hb_sign_fix<<<hb_grid(tot), 256, 0, st>>>(R, k, ldr, Q, m, ldq);
    k_hb_sign_fix_diag<<<hb_grid(k), 256, 0, st>>>(R, k, ldr);
}

void launch_householder_r_blocked(double* S, int64_t m, int64_t k, int64_t lds, double* R,
                                  int64_t ldr, double* ws, size_t wsd, hipStream_t st) {
    hb_factor(S, m, k, lds, R, ldr, nullptr, 0, ws, wsd, st);
}

void launch_householder_qr_blocked(double* S, int64_t m, int64_t k, int64_t lds, double* Q,
                                   int64_t ldq, double* R, int64_t ldr, double* ws, size_t wsd,
                                   hipStream_t st) {
    hb_factor(S, m, k, lds, R, ldr, Q, ldq, ws, wsd, st);
}

}  // namespace rr
