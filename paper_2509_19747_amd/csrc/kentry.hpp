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

}  // namespace rr
