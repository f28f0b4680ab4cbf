// Kernel (Gram) matrix entries for the operators formed on the fly (kernel
// ridge regression, Section 7.2.2): Gaussian RBF and Matern-3/2.
//
// The float32 entry is bitwise symmetric in (i, j).  Callers form
//   s = fl(-0.5 (|x_i|^2 + |x_j|^2)) + sum_k x_ik x_jk
// with the coordinate products added in a fixed order, so s (and K_ij) is the
// same number whichever of the two points is the "row"; then
//   RBF        exp(-kconst r^2) = exp2(c min(s, 0)),   c = fl32(2 kconst log2 e)
//   Matern-3/2 (1 + t) exp(-t),  t = kconst sqrt(max(-2 s, 0)),  c = fl32(kconst)
// using -2 s = r^2.  The float64 entry works on the difference form r^2 directly.
#pragma once
#include "common.hpp"

namespace rr {

constexpr float LOG2E_F = 1.4426950408889634f;

template <int KIND>
RR_DEV float kval32(float s, float c) {
    if (KIND == 1) {
        return __builtin_amdgcn_exp2f(c * fminf(s, 0.0f));
    } else {
        const float t = c * __builtin_sqrtf(fmaxf(-2.0f * s, 0.0f));
        return (1.0f + t) * __builtin_amdgcn_exp2f(-t * LOG2E_F);
    }
}

// s starting value for the pair (i, j) from the row's -|x_i|^2/2 and |x_j|^2.
RR_DEV float kpair_init(float mhalf_ni, float nj) { return fmaf(-0.5f, nj, mhalf_ni); }

template <int KIND>
RR_DEV double kval64(double r2, double kconst) {
    r2 = r2 > 0.0 ? r2 : 0.0;
    if (KIND == 1) return exp(-kconst * r2);
    const double t = kconst * sqrt(r2);
    return (1.0 + t) * exp(-t);
}

// The float32 constant c of kval32 for an operator (kind 1 = RBF, 2 = Matern-3/2).
inline float kernel_c32(int kind, double kconst) {
    return kind == 1 ? (float)(2.0 * kconst * 1.4426950408889634074) : (float)kconst;
}

// 2^t for t <= 0 is table-driven (Tang, ACM TOMS 15(2), 1989): t = m + j/256 + f
// with |f| <= 1/512, 2^t = 2^m 2^(j/256) exp(f ln 2); the last factor is its Taylor
// polynomial of degree 4 (truncation below 4e-17 for |f ln 2| <= ln 2 / 512) and
// 2^(j/256) comes from a 256-entry LDS table (EXP2_TAB entries, filled by
// exp2_table_fill).  About 2 ulp in all.
constexpr double LN2_D = 0.69314718055994530942;
constexpr double LOG2E_D = 1.44269504088896340736;
constexpr int EXP2_TAB = 256;

// Fills tab[0..EXP2_TAB) with 2^(j/256); the caller synchronises before use.
RR_DEV void exp2_table_fill(double* tab) {
    for (int j = threadIdx.x; j < EXP2_TAB; j += blockDim.x) tab[j] = exp2((double)j / EXP2_TAB);
}

RR_DEV double exp2_nonpos(double t, const double* __restrict__ tab) {
    t = fmax(t, -1100.0);
    const double kf = rint(t * EXP2_TAB);
    const double f = fma(kf, -1.0 / EXP2_TAB, t);
    const int k = (int)kf;
    const int j = k & (EXP2_TAB - 1);
    const int m = k >> 8;   // floor(k / 256)
    const double z = f * LN2_D;
    double p = fma(z, 1.0 / 24.0, 1.0 / 6.0);
    p = fma(z, p, 0.5);
    p = fma(z, p, 1.0);
    p = fma(z, p, 1.0);
    return ldexp(tab[j] * p, m);
}

template <int KIND>
RR_DEV double kentry64(double t, double kconst, const double* __restrict__ tab) {
    if (KIND == 1) return exp2_nonpos(t, tab);
    const double kr = kconst * sqrt(fmax(-2.0 * t, 0.0));
    return (1.0 + kr) * exp2_nonpos(-kr * LOG2E_D, tab);
}

}  // namespace rr
