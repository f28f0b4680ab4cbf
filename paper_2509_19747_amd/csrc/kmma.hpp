// Kernel entries from bf16 MFMA: augmented point records whose product is the
// exponent of an entry of the RBF or Matern-3/2 kernel (Section 7.2.2 operators).
//
// The exponent of an entry is one inner product of augmented point records:
//   row    a_i = [g x_i, -g |x_i|^2 / 2, 1]
//   column b_j = [x_j,   1, -g |x_j|^2 / 2]
//   a_i . b_j = g (x_i . x_j - |x_i|^2 / 2 - |x_j|^2 / 2) = -g |x_i - x_j|^2 / 2
// with g = c = 2 kconst log2(e) for the RBF kernel, so K_ij = exp2(a_i . b_j),
// and g = 1 for Matern-3/2, where the product is s_ij of kval32.
//
// Float32 accuracy on bf16 MFMA: every float32 term v splits exactly into three
// bf16 pieces v = v0 + v1 + v2 (each piece rounds the remainder of the previous
// ones to 8 significant bits; 24 bits in all).  A product x y is then the six
// piece products with a + b <= 2 (x0 y0, x0 y1, x1 y0, x0 y2, x1 y1, x2 y0); the
// three dropped ones are below 2^-24 |x y|.  Each piece product is exact in
// float32 and v_mfma_f32_32x32x16_bf16 adds them in float32, so the exponent
// carries float32-class rounding.  The record terms are laid out as six segments
// of DM coordinates (the piece pairs above), then the two augmented terms as
// [p0, p1, p2, 1, 1, 1] x [1, 1, 1, q0, q1, q2], then zeros: 6 DM + 6 terms in
// KB steps of 16.
//
// MFMA layout (v_mfma_f32_32x32x16_bf16): lane l supplies A[row l%32][k 8(l/32) ..
// 8(l/32)+7] and B[k 8(l/32) .. +7][col l%32] of a 16-deep step; accumulator
// element e of lane l is row 8(e/4) + 4(l/32) + (e%4), column l%32.
#pragma once
#include "common.hpp"
#include "kentry.hpp"

namespace rr {

typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <int DM>
struct KmmaShape {
    static constexpr int KT = 6 * DM + 6;       // record terms
    static constexpr int KB = (KT + 15) / 16;   // MFMA steps
    static constexpr int BSTR = 16 * KB + 8;    // LDS stride (bf16) of a column record (padded
                                                // by 16 bytes against bank conflicts)
};

// Piece of x (row side) and of y (column side) in segment seg.
constexpr int kmma_apiece(int seg) { return seg == 2 || seg == 4 ? 1 : seg == 5 ? 2 : 0; }
constexpr int kmma_bpiece(int seg) { return seg == 1 || seg == 4 ? 1 : seg == 3 ? 2 : 0; }

// Exact split v = p[0] + p[1] + p[2] into bf16 pieces (normal-range v).
RR_DEV void kmma_split3(float v, __bf16 (&p)[3]) {
    p[0] = (__bf16)v;
    const float r1 = v - (float)p[0];
    p[1] = (__bf16)r1;
    p[2] = (__bf16)(r1 - (float)p[1]);
}

// Coordinates of a point that half h of a wave needs for its record chunks: for
// DM >= 16, xr[8 m + t] = coordinate 16 m + 8 h + t; otherwise all DM coordinates.
template <int DM>
constexpr int kmma_ncoord() { return DM >= 16 ? DM / 2 : DM; }

template <int DM>
RR_DEV void kmma_coords(const float* __restrict__ rec, int h, float (&xr)[kmma_ncoord<DM>()]) {
    if constexpr (DM >= 16) {
#pragma unroll
        for (int m = 0; m < DM / 16; ++m) {
            const float4 a = *reinterpret_cast<const float4*>(rec + 16 * m + 8 * h);
            const float4 b = *reinterpret_cast<const float4*>(rec + 16 * m + 8 * h + 4);
            xr[8 * m] = a.x; xr[8 * m + 1] = a.y; xr[8 * m + 2] = a.z; xr[8 * m + 3] = a.w;
            xr[8 * m + 4] = b.x; xr[8 * m + 5] = b.y; xr[8 * m + 6] = b.z; xr[8 * m + 7] = b.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < DM; ++k) xr[k] = rec[k];
    }
}

// The KB record chunks (8 terms each) that half h of a wave supplies for one
// point: terms kk = 16 s + 8 h + t, t < 8, of step s.  ROW: the row record
// (coordinates scaled by g, augmented terms [p0, p1, p2, 1, 1, 1]); otherwise the
// column record (augmented terms [1, 1, 1, q0, q1, q2]).  xr: the coordinates of
// kmma_coords; sq: the point's squared norm; emit(s, chunk) receives the chunks
// in order.
template <int DM, bool ROW, typename Emit>
RR_DEV void kmma_record_x(const float (&xr)[kmma_ncoord<DM>()], float sq, float g, int h, Emit&& emit) {
    constexpr int KB = KmmaShape<DM>::KB;
    const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
    __bf16 pa[3];
    kmma_split3(-0.5f * g * sq, pa);
    auto aug = [&](int ka) {   // augmented term ka >= 0 (past the six segments)
        if (ka >= 6) return zero;
        if (ROW) return ka < 3 ? pa[ka] : one;
        return ka < 3 ? one : pa[ka - 3];
    };
    auto piece = [&](int seg) { return ROW ? kmma_apiece(seg) : kmma_bpiece(seg); };
    if constexpr (DM >= 16) {
        // step s covers segment 16 s / DM, coordinates (16 s) % DM + 8 h + t
        __bf16 pc[DM / 16][8][3];
#pragma unroll
        for (int m = 0; m < DM / 16; ++m)
#pragma unroll
            for (int t = 0; t < 8; ++t) kmma_split3(ROW ? g * xr[8 * m + t] : xr[8 * m + t], pc[m][t]);
#pragma unroll
        for (int s = 0; s < KB; ++s) {
            bf16x8_t o;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (16 * s < 6 * DM) o[t] = pc[(16 * s % DM) / 16][t][piece(16 * s / DM)];
                else o[t] = h == 0 ? aug(16 * s + t - 6 * DM) : zero;
            }
            emit(s, o);
        }
    } else {
        __bf16 pc[DM][3];
#pragma unroll
        for (int k = 0; k < DM; ++k) kmma_split3(ROW ? g * xr[k] : xr[k], pc[k]);
        auto val = [&](int kk) { return kk < 6 * DM ? pc[kk % DM][piece(kk / DM)] : aug(kk - 6 * DM); };
#pragma unroll
        for (int s = 0; s < KB; ++s) {
            bf16x8_t o;
#pragma unroll
            for (int t = 0; t < 8; ++t) o[t] = h ? val(16 * s + 8 + t) : val(16 * s + t);
            emit(s, o);
        }
    }
}

// Same, from the point's record rec (DM floats).
template <int DM, bool ROW, typename Emit>
RR_DEV void kmma_record(const float* __restrict__ rec, float sq, float g, int h, Emit&& emit) {
    float xr[kmma_ncoord<DM>()];
    kmma_coords<DM>(rec, h, xr);
    kmma_record_x<DM, ROW>(xr, sq, g, h, emit);
}

// Entry from the record product t (see above).
template <int KIND>
RR_DEV float kmma_entry(float t, float c) {
    // t is -g r^2 / 2 <= 0 up to rounding; near-coincident points may round to a
    // tiny positive t and give an entry a few ulps above 1
    if (KIND == 1) return __builtin_amdgcn_exp2f(t);
    return kval32<2>(t, c);
}

}  // namespace rr
