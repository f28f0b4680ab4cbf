// Small dense float64 factorizations kept on the device (no host round trip):
//  * blocked upper Cholesky A = R^T R (Algorithm chol_qr / prec_chol_qr step
//    "chol", the core factor R_Omega); failure is reported in a device status
//    word, which the host reads once to drive the shift ladder;
//  * Householder QR (R only, or R and explicit Q) for the sketched factor
//    R_sk = qr(Theta A_mu Omega) and the 2l x l reduced QR of the joint basis
//    (Section 5.1), with the diagonal of R made positive;
//  * inverse of an upper-triangular matrix (applied with a GEMM afterwards).
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <type_traits>

namespace rr {

// ============================================================== Cholesky
constexpr int CH_NB = 32;

// One block row of the blocked Cholesky in a single launch of 64-thread blocks:
// every block factors the kb x kb diagonal block A11 = R11^T R11 (identical
// arithmetic in every block), then solves R11^T X = A12 for its 64 columns of the
// row panel.  Lane j holds column j of A11 in registers; row k of R11 is shared
// through LDS once it is formed, so the inner loops only read LDS broadcasts.
// Block 0 writes R11 back (zeros below the diagonal) and raises the status word
// when a pivot is not positive and finite.
__global__ __launch_bounds__(64) void k_chol_panel(double* A, int64_t lda, int kb, int64_t rest,
                                                   int32_t* status) {
    __shared__ double rk[CH_NB][CH_NB + 1];   // rk[k][i] = R11(k, i), i >= k
    if (*status) return;
    const int t = threadIdx.x;
    double col[CH_NB];
#pragma unroll
    for (int i = 0; i < CH_NB; ++i)
        col[i] = (t < kb && i <= t) ? A[i + (int64_t)t * lda] : 0.0;
    const int64_t jc = (int64_t)blockIdx.x * 64 + t;   // panel column of this thread
    double x[CH_NB];
#pragma unroll
    for (int i = 0; i < CH_NB; ++i) x[i] = (jc < rest && i < kb) ? A[i + (kb + jc) * lda] : 0.0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < CH_NB; ++k) {
        if (k >= kb) continue;   // uniform
        const double dkk = __shfl(col[k], k);
        const bool ok = dkk > 0.0 && isfinite(dkk);
        bad = bad || !ok;
        const double piv = ok ? sqrt(dkk) : 1.0;
        const double rkt = (t == k) ? piv : (t > k ? col[k] / piv : 0.0);
        if (t >= k) col[k] = rkt;
        if (t < CH_NB) rk[k][t] = rkt;
        __syncthreads();
#pragma unroll
        for (int i = k + 1; i < CH_NB; ++i) {
            const double rki = rk[k][i];
            if (i <= t && t < kb) col[i] = fma(-rki, rkt, col[i]);
        }
    }
    __syncthreads();
    if (jc < rest) {
#pragma unroll
        for (int i = 0; i < CH_NB; ++i) {
            if (i >= kb) continue;
            double s = x[i];
#pragma unroll
            for (int k = 0; k < i; ++k) s = fma(-rk[k][i], x[k], s);
            x[i] = s / rk[i][i];
        }
#pragma unroll
        for (int i = 0; i < CH_NB; ++i)
            if (i < kb) A[i + (kb + jc) * lda] = x[i];
    }
    if (blockIdx.x == 0) {
        if (t < kb)
#pragma unroll
            for (int i = 0; i < CH_NB; ++i)
                if (i < kb) A[i + (int64_t)t * lda] = (i <= t) ? col[i] : 0.0;
        if (t == 0 && bad) *status = 1;
    }
}

void launch_cholesky_upper(double* A, int64_t l, int64_t lda, int32_t* status, double* ws,
                           size_t ws_doubles, hipStream_t st) {
    for (int64_t k0 = 0; k0 < l; k0 += CH_NB) {
        const int kb = (int)((l - k0 < CH_NB) ? l - k0 : CH_NB);
        double* A11 = A + k0 + k0 * lda;
        const int64_t rest = l - k0 - kb;
        k_chol_panel<<<(unsigned)std::max<int64_t>((rest + 63) / 64, 1), 64, 0, st>>>(A11, lda, kb, rest,
                                                                                     status);
        if (rest > 0) {
            const double* A12 = A + k0 + (k0 + kb) * lda;
            double* A22 = A + (k0 + kb) + (k0 + kb) * lda;
            launch_gemm(DT_F64, true, DT_F64, false, rest, rest, kb, A12, lda, A12, lda, A22, lda,
                        -1.0, 1.0, ws, ws_doubles, st);
        }
    }
    launch_zero_lower(A, l, lda, st);
}

// ============================================================ Householder
constexpr int HH_COLS = 8;
constexpr int HH_THREADS = 256;

// One Householder step on column kc of S (m x k).  Every block rebuilds the
// reflector from column kc (identical arithmetic in every block) and applies it
// to its HH_COLS trailing columns; block 0 writes column kc of R and, if V is
// given, the reflector v and its factor 2/(v^T v).
__global__ __launch_bounds__(HH_THREADS) void k_house_step(double* S, int64_t m, int64_t k,
                                                           int64_t lds, int64_t kc, double* R,
                                                           int64_t ldr, double* V, int64_t ldv,
                                                           double* tauv) {
    extern __shared__ double x[];
    __shared__ double sc[HH_THREADS / WAVE];
    __shared__ double wsh[HH_COLS];
    const int64_t L = m - kc;
    const double* col = S + kc + kc * lds;
    double s1 = 0.0;
    for (int64_t i = threadIdx.x; i < L; i += HH_THREADS) {
        const double v = col[i];
        x[i] = v;
        if (i > 0) s1 = fma(v, v, s1);
    }
    s1 = block_sum(s1, sc);   // includes a barrier after x[] is written
    const double alpha = x[0];
    __syncthreads();   // every thread has read x[0] before it is replaced by v0
    const double normx = sqrt(fma(alpha, alpha, s1));
    const double beta = (alpha >= 0.0) ? -normx : normx;
    const double v0 = alpha - beta;
    const double vtv = fma(v0, v0, s1);
    const double f = (vtv > 0.0) ? 2.0 / vtv : 0.0;
    if (threadIdx.x == 0) x[0] = v0;
    __syncthreads();

    if (blockIdx.x == 0) {
        for (int64_t i = threadIdx.x; i < k; i += HH_THREADS) {
            double rv;
            if (i < kc) rv = S[i + kc * lds];
            else if (i == kc) rv = (normx > 0.0) ? beta : alpha;
            else rv = 0.0;
            R[i + kc * ldr] = rv;
        }
        if (V) {
            for (int64_t i = threadIdx.x; i < m; i += HH_THREADS) V[i + kc * ldv] = (i < kc) ? 0.0 : x[i - kc];
            if (threadIdx.x == 0) tauv[kc] = f;
        }
    }
    if (f == 0.0) return;
    const int64_t jb = kc + 1 + (int64_t)blockIdx.x * HH_COLS;
    double acc[HH_COLS];
#pragma unroll
    for (int c = 0; c < HH_COLS; ++c) acc[c] = 0.0;
    for (int64_t i = threadIdx.x; i < L; i += HH_THREADS) {
        const double xi = x[i];
#pragma unroll
        for (int c = 0; c < HH_COLS; ++c) {
            const int64_t j = jb + c;
            if (j < k) acc[c] = fma(xi, S[kc + i + j * lds], acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < HH_COLS; ++c) {
        const double w = block_sum(acc[c], sc);
        if (threadIdx.x == 0) wsh[c] = w * f;
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < L; i += HH_THREADS) {
        const double xi = x[i];
#pragma unroll
        for (int c = 0; c < HH_COLS; ++c) {
            const int64_t j = jb + c;
            if (j < k) S[kc + i + j * lds] = fma(-wsh[c], xi, S[kc + i + j * lds]);
        }
    }
}

// Make diag(R) positive: rows with a negative diagonal are negated (and the
// matching columns of Q, if given).
__global__ void k_sign_fix(double* R, int64_t k, int64_t ldr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (R[i + i * ldr] < 0.0)
            for (int64_t j = i; j < k; ++j) R[i + j * ldr] = -R[i + j * ldr];
    }
}
__global__ void k_sign_fix_q(const double* R, int64_t k, int64_t ldr, double* Q, int64_t m,
                             int64_t ldq) {
    const int64_t total = m * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, j = e / m;
        if (R[j + j * ldr] < 0.0) Q[i + j * ldq] = -Q[i + j * ldq];
    }
}

static int g256(int64_t total) {
    int64_t g = (total + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

static void householder_r_unblocked(double* S, int64_t m, int64_t k, int64_t lds, double* R,
                                    int64_t ldr, hipStream_t st) {
    const size_t shm = (size_t)m * sizeof(double);
    for (int64_t kc = 0; kc < k; ++kc) {
        const int64_t rest = k - kc - 1;
        const int g = (int)((rest + HH_COLS - 1) / HH_COLS > 0 ? (rest + HH_COLS - 1) / HH_COLS : 1);
        k_house_step<<<g, HH_THREADS, shm, st>>>(S, m, k, lds, kc, R, ldr, nullptr, 0, nullptr);
    }
    k_sign_fix<<<g256(k), 256, 0, st>>>(R, k, ldr);
}

// Q = H_0 ... H_{k-1} [I; 0]: accumulate backwards, one reflector per launch.
__global__ __launch_bounds__(HH_THREADS) void k_house_apply_q(double* Q, int64_t m, int64_t k,
                                                              int64_t ldq, const double* V,
                                                              int64_t ldv, const double* tauv,
                                                              int64_t kc) {
    __shared__ double sc[HH_THREADS / WAVE];
    __shared__ double wsh[HH_COLS];
    const double f = tauv[kc];
    if (f == 0.0) return;
    const int64_t jb = (int64_t)blockIdx.x * HH_COLS;
    double acc[HH_COLS];
#pragma unroll
    for (int c = 0; c < HH_COLS; ++c) acc[c] = 0.0;
    for (int64_t i = kc + threadIdx.x; i < m; i += HH_THREADS) {
        const double vi = V[i + kc * ldv];
#pragma unroll
        for (int c = 0; c < HH_COLS; ++c) {
            const int64_t j = jb + c;
            if (j < k) acc[c] = fma(vi, Q[i + j * ldq], acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < HH_COLS; ++c) {
        const double w = block_sum(acc[c], sc);
        if (threadIdx.x == 0) wsh[c] = w * f;
    }
    __syncthreads();
    for (int64_t i = kc + threadIdx.x; i < m; i += HH_THREADS) {
        const double vi = V[i + kc * ldv];
#pragma unroll
        for (int c = 0; c < HH_COLS; ++c) {
            const int64_t j = jb + c;
            if (j < k) Q[i + j * ldq] = fma(-wsh[c], vi, Q[i + j * ldq]);
        }
    }
}

__global__ void k_eye_rect(double* Q, int64_t m, int64_t k, int64_t ldq) {
    const int64_t total = m * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, j = e / m;
        Q[i + j * ldq] = (i == j) ? 1.0 : 0.0;
    }
}

static void householder_qr_unblocked(double* S, int64_t m, int64_t k, int64_t lds, double* Q,
                                     int64_t ldq, double* R, int64_t ldr, double* ws, hipStream_t st) {
    double* V = ws;                 // m x k
    double* tauv = ws + m * k;      // k
    const size_t shm = (size_t)m * sizeof(double);
    for (int64_t kc = 0; kc < k; ++kc) {
        const int64_t rest = k - kc - 1;
        const int g = (int)((rest + HH_COLS - 1) / HH_COLS > 0 ? (rest + HH_COLS - 1) / HH_COLS : 1);
        k_house_step<<<g, HH_THREADS, shm, st>>>(S, m, k, lds, kc, R, ldr, V, m, tauv);
    }
    k_eye_rect<<<g256(m * k), 256, 0, st>>>(Q, m, k, ldq);
    const int gq = (int)((k + HH_COLS - 1) / HH_COLS);
    for (int64_t kc = k - 1; kc >= 0; --kc)
        k_house_apply_q<<<gq, HH_THREADS, 0, st>>>(Q, m, k, ldq, V, m, tauv, kc);
    k_sign_fix_q<<<g256(m * k), 256, 0, st>>>(R, k, ldr, Q, m, ldq);
    k_sign_fix<<<g256(k), 256, 0, st>>>(R, k, ldr);
}

// Blocked panels when the panel fits the register layout (m <= 2048), one
// reflector per launch otherwise.
void launch_householder_r(double* S, int64_t m, int64_t k, int64_t lds, double* R, int64_t ldr,
                          double* ws, size_t wsd, hipStream_t st) {
    if (householder_blocked_ok(m, k) && wsd >= householder_ws_doubles(m, k))
        launch_householder_r_blocked(S, m, k, lds, R, ldr, ws, wsd, st);
    else
        householder_r_unblocked(S, m, k, lds, R, ldr, st);
}
void launch_householder_qr(double* S, int64_t m, int64_t k, int64_t lds, double* Q, int64_t ldq,
                           double* R, int64_t ldr, double* ws, size_t wsd, hipStream_t st) {
    if (householder_blocked_ok(m, k) && wsd >= householder_ws_doubles(m, k))
        launch_householder_qr_blocked(S, m, k, lds, Q, ldq, R, ldr, ws, wsd, st);
    else
        householder_qr_unblocked(S, m, k, lds, Q, ldq, R, ldr, ws, st);
}

// ==================================================== triangular inverse
// Column j of X = R^{-1}: column-oriented back substitution on e_j.
__global__ __launch_bounds__(256) void k_tri_inv_upper(const double* R, int64_t l, int64_t ldr,
                                                       double* X, int64_t ldx) {
    extern __shared__ double xs[];
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i <= j; i += blockDim.x) xs[i] = (i == j) ? 1.0 : 0.0;
    __syncthreads();
    for (int64_t i = j; i >= 0; --i) {
        const double xi = xs[i] / R[i + i * ldr];
        __syncthreads();
        if (threadIdx.x == 0) xs[i] = xi;
        for (int64_t r = threadIdx.x; r < i; r += blockDim.x) xs[r] = fma(-R[r + i * ldr], xi, xs[r]);
        __syncthreads();
    }
    for (int64_t i = threadIdx.x; i < l; i += blockDim.x) X[i + j * ldx] = (i <= j) ? xs[i] : 0.0;
}

// One wave per column j of X = R^{-1}, for l <= 64 U: lane t holds rows t + 64 u
// (u < U) of the column in registers.  Back substitution from row j up: row r's
// value is final once the rows below it are done; the wave reads it from its lane
// (readlane), scales it by 1 / R_rr and subtracts its multiple of column r of R
// from the rows above it, so a step's dependency chain is a readlane, a multiply
// and an FMA.  Everything else is kept off that chain: the columns of R come in
// panels of CP columns through LDS (two buffers), each panel's global loads issued
// two panels before its steps run (two register sets), the panel's LDS reads
// issued together before its steps, and 1 / R_rr formed per panel in parallel.
RR_DEV double tri_readlane(double x, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int U, int CP>
__global__ __launch_bounds__(64) void k_tri_inv_upper_wave(const double* __restrict__ R, int64_t l,
                                                           int64_t ldr, double* __restrict__ X,
                                                           int64_t ldx) {
    static_assert(64 % (2 * CP) == 0, "a slot holds an even number of panels");
    constexpr int LR = 64 * U;       // LDS rows per staged column
    extern __shared__ double rs[];   // 2 buffers x CP columns x LR rows
    const int lane = threadIdx.x;
    const int j = (int)blockIdx.x;
    const int uj = j >> 6;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (64 * u + lane == j) ? 1.0 : 0.0;
    // panel p = columns p CP + c (c < CP), entries at rows <= the column; columns
    // past j (and panels p < 0) load as zeros and their steps are skipped
    double ga[CP][U], gb[CP][U];
    // The loads are unconditional (clamped addresses, masked values): no branches
    // around them, so the wait before staging a panel covers only that panel's
    // loads and not the ones just issued for the panel after it.
    auto gload = [&](int p, double (&g)[CP][U]) {
#pragma unroll
        for (int c = 0; c < CP; ++c) {
            const int r = p * CP + c;
            const int rc = r < 0 ? 0 : (r > j ? j : r);
#pragma unroll
            for (int w = 0; w < U; ++w) {
                const int i = 64 * w + lane;
                const double x = R[(i < rc ? i : rc) + (int64_t)rc * ldr];
                g[c][w] = (r >= 0 && r <= j && i <= r) ? x : 0.0;
            }
        }
    };
    auto lstore = [&](int p, const double (&g)[CP][U]) {
        double* dst = rs + (p & 1) * CP * LR;
#pragma unroll
        for (int c = 0; c < CP; ++c)
#pragma unroll
            for (int w = 0; w < U; ++w) dst[c * LR + 64 * w + lane] = g[c][w];
    };
    // the steps of panel p (rows of slot u), its columns read from LDS
    auto steps = [&](int p, auto uc) {
        constexpr int u = decltype(uc)::value;
        const double* Rb = rs + (p & 1) * CP * LR;
        const int rlo = p * CP;
        double col[CP][u + 1];
#pragma unroll
        for (int c = 0; c < CP; ++c)
#pragma unroll
            for (int w = 0; w <= u; ++w) col[c][w] = Rb[c * LR + 64 * w + lane];
        const double dinv = lane < CP ? 1.0 / Rb[lane * LR + rlo + lane] : 0.0;
#pragma unroll
        for (int c = CP - 1; c >= 0; --c) {
            const int r = rlo + c;
            if (r > j) continue;   // uniform over the wave
            const int rr = r - 64 * u;
            const double xr = tri_readlane(v[u], rr) * tri_readlane(dinv, c);
            if (lane == rr) v[u] = xr;
#pragma unroll
            for (int w = 0; w < u; ++w) v[w] = fma(-col[c][w], xr, v[w]);
            if (lane < rr) v[u] = fma(-col[c][u], xr, v[u]);
        }
    };
    // panel p's steps with panel p - 1 in flight in `hold`: load p - 2 into `free`,
    // run p, then stage p - 1 (its buffer was last read before the previous barrier)
    auto panel = [&](int p, auto uc, double (&hold)[CP][U], double (&free)[CP][U]) {
        gload(p - 2, free);
        steps(p, uc);
        lstore(p - 1, hold);
        __syncthreads();
    };
    // slot uj starts at an even panel count from its bottom (a leading panel past j
    // is empty), so every slot runs whole pairs and the register roles line up
    const int ppb = 64 / CP;                          // panels per slot
    int p0 = uj * ppb + ((j - 64 * uj) / CP | 1);     // odd offset within the slot
    gload(p0, ga);
    lstore(p0, ga);
    gload(p0 - 1, ga);
    __syncthreads();
    auto slot = [&](auto uc) {
        constexpr int u = decltype(uc)::value;
        if (u > uj) return;
        const int ptop = (u == uj) ? p0 : u * ppb + ppb - 1;
        for (int p = ptop; p >= u * ppb; p -= 2) {
            panel(p, uc, ga, gb);
            panel(p - 1, uc, gb, ga);
        }
    };
    [&] {
        auto down = [&](auto self, auto uc) -> void {
            constexpr int u = decltype(uc)::value;
            slot(uc);
            if constexpr (u > 0) self(self, std::integral_constant<int, u - 1>{});
        };
        down(down, std::integral_constant<int, U - 1>{});
    }();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = 64 * u + lane;
        if (i < l) X[i + (int64_t)j * ldx] = (i <= j) ? v[u] : 0.0;
    }
}

template <int U, int CP>
static void tri_inv_wave(const double* R, int64_t l, int64_t ldr, double* X, int64_t ldx, hipStream_t st) {
    const size_t shm = (size_t)2 * CP * 64 * U * sizeof(double);
    k_tri_inv_upper_wave<U, CP><<<(unsigned)l, 64, shm, st>>>(R, l, ldr, X, ldx);
}

void launch_tri_inv_upper(const double* R, int64_t l, int64_t ldr, double* X, int64_t ldx,
                          hipStream_t st) {
    if (l <= 0) return;
    const int64_t slots = (l + 63) / 64;
    if (slots <= 1) tri_inv_wave<1, 4>(R, l, ldr, X, ldx, st);
    else if (slots <= 2) tri_inv_wave<2, 4>(R, l, ldr, X, ldx, st);
    else if (slots <= 4) tri_inv_wave<4, 4>(R, l, ldr, X, ldx, st);
    else if (slots <= 8) tri_inv_wave<8, 4>(R, l, ldr, X, ldx, st);
    else k_tri_inv_upper<<<(unsigned)l, 256, (size_t)l * sizeof(double), st>>>(R, l, ldr, X, ldx);
}

}  // namespace rr
