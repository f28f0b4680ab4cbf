// Largest eigenvalue of a small symmetric positive semidefinite matrix, for the
// tau of eq. nys_tau (tau = 1 / lambda_max(G), G = R^{-T} (Omega^T A_mu Omega) R^{-1}).
//
// Lanczos with full reorthogonalisation in one 1024-thread workgroup:
//   * the current vector v and the work vector w live in LDS, the Lanczos basis
//     V (k x (steps+1)) in global memory;
//   * w = G v reads G column by column (coalesced over the rows), v is an LDS
//     broadcast; two classical Gram-Schmidt passes against all of V follow;
//   * after every step wave 0 brackets the largest eigenvalue theta of the
//     tridiagonal T by multisection (Sturm counts at 64 points per round), and
//     lane 0 bounds the Ritz residual ||G y - theta y|| = beta_j |s_last| with
//     s_last^2 = chi_{j}(theta) / chi'_{j+1}(theta) (chi_m: characteristic
//     polynomial of the leading m x m block of T), which bounds |theta - lambda|.
// The loop ends when that bound is below 1e-14 theta, when beta vanishes (an
// invariant subspace), or after k steps (then T holds the whole spectrum).
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cfloat>

namespace rr {

constexpr int LZ_THREADS = 1024;

// number of eigenvalues of the m x m tridiagonal (a, off-diagonal squares b2) below x
RR_DEV int sturm_below(const double* a, const double* b2, int m, double x, double pivmin) {
    int c = 0;
    double q = a[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    for (int i = 1; i < m; ++i) {
        q = (a[i] - x) - b2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

__global__ __launch_bounds__(LZ_THREADS) void k_lanczos_lmax(const double* __restrict__ G, int64_t ldg,
                                                            int k, uint64_t seed, int mmax,
                                                            double* __restrict__ V, double* out) {
    extern __shared__ double sh[];
    double* v = sh;              // k
    double* w = v + k;           // k
    double* al = w + k;          // mmax   diagonal of T
    double* be = al + mmax;      // mmax   off-diagonal of T (be[j] couples steps j, j+1)
    double* b2 = be + mmax;      // mmax   squares of be
    double* h = b2 + mmax;       // mmax   reorthogonalisation coefficients
    double* sc = h + mmax;       // 16     block-sum scratch
    __shared__ double s_theta, s_res;
    __shared__ int s_stop;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = LZ_THREADS / 64;

    double s = 0.0;
    for (int i = t; i < k; i += LZ_THREADS) {
        const double g = gauss_at(seed, (uint64_t)i);
        w[i] = g;
        s = fma(g, g, s);
    }
    s = block_sum(s, sc);
    const double inv0 = 1.0 / sqrt(s);
    for (int i = t; i < k; i += LZ_THREADS) {
        v[i] = w[i] * inv0;
        V[i] = v[i];
    }
    if (t == 0) { s_theta = 0.0; s_res = INFINITY; s_stop = 0; }
    __syncthreads();
    int steps = 0;
    for (int j = 0; j < mmax; ++j) {
        for (int i = t; i < k; i += LZ_THREADS) {
            double acc = 0.0;
            for (int c = 0; c < k; ++c) acc = fma(G[i + (int64_t)c * ldg], v[c], acc);
            w[i] = acc;
        }
        __syncthreads();
        double p = 0.0;
        for (int i = t; i < k; i += LZ_THREADS) p = fma(v[i], w[i], p);
        double a = block_sum(p, sc);
        const double bprev = j > 0 ? be[j - 1] : 0.0;
        for (int i = t; i < k; i += LZ_THREADS) {
            double x = fma(-a, v[i], w[i]);
            if (j > 0) x = fma(-bprev, V[i + (int64_t)(j - 1) * k], x);
            w[i] = x;
        }
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = wave; q <= j; q += nw) {
                double dsum = 0.0;
                for (int i = lane; i < k; i += 64) dsum = fma(V[i + (int64_t)q * k], w[i], dsum);
                dsum = wave_sum(dsum);
                if (lane == 0) h[q] = dsum;
            }
            __syncthreads();
            for (int i = t; i < k; i += LZ_THREADS) {
                double x = w[i];
                for (int q = 0; q <= j; ++q) x = fma(-h[q], V[i + (int64_t)q * k], x);
                w[i] = x;
            }
            if (pass == 0) a += h[j];
            __syncthreads();
        }
        p = 0.0;
        for (int i = t; i < k; i += LZ_THREADS) p = fma(w[i], w[i], p);
        const double bn = sqrt(block_sum(p, sc));
        if (t == 0) {
            al[j] = a;
            be[j] = bn;
            b2[j] = bn * bn;
        }
        __syncthreads();
        steps = j + 1;
        const int m = j + 1;
        if (wave == 0) {
            // bracket lambda_max(T_m): Gershgorin above, the previous Ritz value below
            double hi = -INFINITY, bmax2 = 0.0, lo = INFINITY;
            for (int i = 0; i < m; ++i) {
                const double r = (i > 0 ? be[i - 1] : 0.0) + (i + 1 < m ? be[i] : 0.0);
                hi = fmax(hi, al[i] + r);
                lo = fmin(lo, al[i] - r);
                if (i + 1 < m) bmax2 = fmax(bmax2, b2[i]);
            }
            if (j > 0) lo = fmax(lo, s_theta - 4.0 * DBL_EPSILON * fabs(s_theta));
            const double pivmin = DBL_MIN * fmax(1.0, bmax2);
            for (int round = 0; round < 24 && hi - lo > 2.0 * DBL_EPSILON * fabs(hi); ++round) {
                const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
                const bool above = sturm_below(al, b2, m, x, pivmin) == m;
                const uint64_t bal = __ballot(above);
                const int f = bal ? __builtin_ctzll(bal) : 64;
                const double xf = lo + (hi - lo) * (double)(f + 1) / 65.0;
                const double xp = lo + (hi - lo) * (double)f / 65.0;
                if (f < 64) hi = xf;
                lo = f > 0 ? xp : lo;
            }
            const double theta = 0.5 * (lo + hi);
            if (lane == 0) {
                // s_last^2 = chi_{m-1}(theta) / chi'_m(theta), uniformly rescaled recurrences
                double P0 = 1.0, P1 = theta - al[0], D0 = 0.0, D1 = 1.0;
                for (int q = 1; q < m; ++q) {
                    const double P2 = (theta - al[q]) * P1 - b2[q - 1] * P0;
                    const double D2 = P1 + (theta - al[q]) * D1 - b2[q - 1] * D0;
                    P0 = P1; P1 = P2; D0 = D1; D1 = D2;
                    const double mag = fabs(P1) + fabs(D1) + fabs(P0) + fabs(D0);
                    if (mag > 1e150 || (mag < 1e-150 && mag > 0.0)) {
                        const double f = 1.0 / mag;
                        P0 *= f; P1 *= f; D0 *= f; D1 *= f;
                    }
                }
                const double ratio = (D1 != 0.0) ? P0 / D1 : INFINITY;
                const double res = bn * sqrt(fmax(ratio, 0.0));
                s_theta = theta;
                s_res = (ratio >= 0.0 && isfinite(ratio)) ? res : bn;
                s_stop = (s_res <= 1e-14 * theta) || (bn <= DBL_EPSILON * theta) || (m >= k);
            }
        }
        __syncthreads();
        if (s_stop || j + 1 >= mmax) break;
        const double inv = 1.0 / bn;
        for (int i = t; i < k; i += LZ_THREADS) {
            const double x = w[i] * inv;
            v[i] = x;
            V[i + (int64_t)(j + 1) * k] = x;
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = s_theta;
        out[1] = s_res;
        out[2] = (double)steps;
    }
}

int lanczos_max_dim() { return 1536; }

size_t lanczos_ws_doubles(int64_t k) {
    const int64_t mmax = std::min<int64_t>(k, 1024);
    return (size_t)k * (size_t)(mmax + 1);
}

void launch_lanczos_lmax(const double* G, int64_t ldg, int64_t k, uint64_t seed, double* ws, double* out3,
                         hipStream_t st) {
    const int mmax = (int)std::min<int64_t>(k, 1024);
    const size_t lds = ((size_t)2 * k + 4 * (size_t)mmax + 16) * sizeof(double);
    k_lanczos_lmax<<<1, LZ_THREADS, lds, st>>>(G, ldg, (int)k, seed, mmax, ws, out3);
}

}  // namespace rr
