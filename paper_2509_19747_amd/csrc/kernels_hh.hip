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
// The trailing columns are then updated with three GEMMs,
//   W = V^T S_t,  W <- T^T W,  S_t <- S_t - V W,
// and an explicit Q is accumulated backwards panel by panel with
//   W = V^T Q_t,  W <- T W,  Q_t <- Q_t - V W.
// Each reflector is H = I - f v v^T with v_0 = alpha - beta, beta = -sign(alpha)
// ||x|| and f = 2 / v^T v (Golub and Van Loan, Algorithm 5.1.1, unnormalised).
// R's diagonal is made positive at the end (R <- D R, Q <- Q D with D = sign).
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>

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
    __shared__ double red[HB_WAVES * NB];
    __shared__ double tot[NB];
    __shared__ double Tsh[NB * NB];
    __shared__ double s_alpha;
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

    for (int c = 0; c < nbe; ++c) {
        const int64_t kc = j0 + c;
        // x = column c at rows >= kc; the pivot row kc is thread c, register row 0
        double s1[1] = {0.0};
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
            double x = 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q == c) x = a[r][q];
            if (i > kc && i < m) s1[0] = fma(x, x, s1[0]);
            if (i == kc) s_alpha = x;
        }
        hb_block_sum<1>(s1, red, tot);   // barriers also publish s_alpha
        const double alpha = s_alpha;
        const double normx = sqrt(fma(alpha, alpha, s1[0]));
        const double beta = (alpha >= 0.0) ? -normx : normx;
        const double v0 = alpha - beta;
        const double vtv = fma(v0, v0, s1[0]);
        const double f = (vtv > 0.0) ? 2.0 / vtv : 0.0;
        // R entries of column kc: rows [j0, kc) from the panel, the diagonal, zeros below
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
            double x = 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q == c) x = a[r][q];
            if (i < kc) R[i + kc * ldr] = x;
            else if (i == kc) R[i + kc * ldr] = (normx > 0.0) ? beta : alpha;
            else if (i < k) R[i + kc * ldr] = 0.0;
        }
        // v into column c (zeros above the pivot)
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t i = j0 + t + (int64_t)HB_THREADS * r;
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q == c) a[r][q] = (i < kc || i >= m) ? 0.0 : (i == kc ? v0 : a[r][q]);
        }
        // dots of v with every panel column: previous reflectors (for T) and the
        // columns still to be reduced (for the update)
        double dots[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) dots[q] = 0.0;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q == c) v = a[r][q];
#pragma unroll
            for (int q = 0; q < NB; ++q) dots[q] = fma(v, a[r][q], dots[q]);
        }
        hb_block_sum<NB>(dots, red, tot);
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q == c) v = a[r][q];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q > c && q < nbe) a[r][q] = fma(-f * dots[q], v, a[r][q]);
        }
        // T(:, c): T(c, c) = f, T(0:c, c) = -f T(0:c, 0:c) (V(:, 0:c)^T v); thread i
        // forms row i (it reads only columns < c, which no thread writes now)
        if (t < c) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j >= t && j < c) s = fma(Tsh[t + j * NB], dots[j], s);
            Tsh[t + c * NB] = -f * s;
        } else if (t == c) {
            Tsh[c + c * NB] = f;
            tauv[kc] = f;
        }
        __syncthreads();
    }
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
    const size_t base = (size_t)m * k + k + (size_t)panels * HB_NB * HB_NB + 2 * (size_t)HB_NB * k;
    return base + gemm_ws_doubles(HB_NB, k, m) + 64;
}

bool householder_blocked_ok(int64_t m, int64_t k) { return m <= 4 * HB_THREADS && k >= 1 && m >= k; }

template <int RR, int NB>
static void hb_panel(double* S, int64_t m, int64_t k, int64_t lds, int64_t j0, int nbe, double* V,
                     double* tauv, double* T, double* R, int64_t ldr, hipStream_t st) {
    k_panel_qr<RR, NB><<<1, HB_THREADS, 0, st>>>(S, m, k, lds, j0, nbe, V, m, tauv, T, R, ldr);
}

// Shared driver: factor S panel by panel, update the trailing columns; when Q is
// given, accumulate it afterwards.  Panels of 16 columns while the panel rows
// fit 2 registers per thread, 8 columns beyond (4 rows per thread).
// ws: householder_ws_doubles(m, k).
static void hb_factor(double* S, int64_t m, int64_t k, int64_t lds, double* R, int64_t ldr,
                      double* Q, int64_t ldq, double* ws, size_t wsd, hipStream_t st) {
    const int nb = m <= 2 * HB_THREADS ? 16 : 8;
    double* V = ws;
    double* tauv = V + (size_t)m * k;
    double* Tall = tauv + k;
    const int64_t panels = (k + nb - 1) / nb;
    double* W = Tall + (size_t)panels * nb * nb;
    double* W2 = W + (size_t)nb * k;
    double* gws = W2 + (size_t)nb * k;
    const size_t gwsd = wsd - (size_t)(gws - ws);
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
            const double* Vp = V + j0 + j0 * m;
            double* St = S + j0 + jt * lds;
            // W = Vp^T S_t (nbe x nt); W2 = T^T W; S_t -= Vp W2
            launch_gemm(DT_F64, true, DT_F64, false, nbe, nt, L, Vp, m, St, lds, W, nb, 1.0, 0.0, gws,
                        gwsd, st);
            launch_gemm(DT_F64, true, DT_F64, false, nbe, nt, nbe, T, nb, W, nb, W2, nb, 1.0, 0.0, gws,
                        gwsd, st);
            launch_gemm(DT_F64, false, DT_F64, false, L, nt, nbe, Vp, m, W2, nb, St, lds, -1.0, 1.0, gws,
                        gwsd, st);
        }
    }
    if (Q) {
        // Q = [I; 0], then Q_t <- Q_t - Vp (T (Vp^T Q_t)) for panels in reverse
        k_hb_eye<<<hb_grid(m * k), 256, 0, st>>>(Q, m, k, ldq);
        for (int64_t p = panels - 1; p >= 0; --p) {
            const int64_t j0 = p * nb;
            const int nbe = (int)std::min<int64_t>(nb, k - j0);
            const double* T = Tall + (size_t)p * nb * nb;
            const int64_t L = m - j0, nt = k - j0;
            const double* Vp = V + j0 + j0 * m;
            double* Qt = Q + j0 + j0 * ldq;
            launch_gemm(DT_F64, true, DT_F64, false, nbe, nt, L, Vp, m, Qt, ldq, W, nb, 1.0, 0.0, gws,
                        gwsd, st);
            launch_gemm(DT_F64, false, DT_F64, false, nbe, nt, nbe, T, nb, W, nb, W2, nb, 1.0, 0.0, gws,
                        gwsd, st);
            launch_gemm(DT_F64, false, DT_F64, false, L, nt, nbe, Vp, m, W2, nb, Qt, ldq, -1.0, 1.0, gws,
                        gwsd, st);
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
