// Kernel sketch on bf16 MFMA: Y = scale * K Omega + mu Omega (the sketch
// A_mu Omega of Algorithm RandRAND_PCG, step 2, for a kernel operator in
// float32 mode).  Omega's entries are exact in bf16 (SRHT +-1, or a Gaussian
// drawn in bf16); each float32 kernel entry is split into hi = bf16(k) and
// lo = bf16(k - hi) (about 16 significant bits together) and both parts go
// through v_mfma_f32_32x32x16_bf16 with float32 accumulation.
//
// Block: 512 threads = 8 waves, tile 128 rows x 512 columns (l <= 512 in one
// column tile, so every kernel entry is formed once per row tile); wave w owns
// rows 64*(w&1)..+63 and columns 128*((w>>1)&3)..+127 (2 x 4 MFMA tiles of
// 32 x 32).  Per step of 32 points the block forms the 128 x 32 kernel tile and
// stages the 32 x 512 slice of Omega in LDS (thread t: column t, loaded into
// registers up to three steps ahead).  The kernel tile is formed on the matrix cores too:
// waves 0-3 each form one 32 x 32 quarter as the product of augmented point
// records (kmma.hpp: float32-class exponents from three-piece bf16 splits), then
// exp2 and the hi/lo split on the vector ALU.  The records of the block's rows
// are built once into LDS; those of the step's points are built by the forming
// lanes from coordinates loaded one step ahead.  The tiles are double-buffered:
// a step's product MFMAs read one buffer while waves 0-3 form the next step into
// the other, so each SIMD pairs a forming wave (formation first, then its product
// MFMAs) with a wave that only multiplies.
// The point range may be split over several blocks (split-K) to fill the GPU
// evenly; partial sums then go to a workspace and a second kernel adds them in a
// fixed order.  The MFMA operands use one consistent k order for A and B (lane l
// holds k = 8*(l/32) .. +7 of a 16-point half step), which is all the product
// needs.  Accumulator element j of lane l is row 8*(j/4) + 4*(l/32) + (j%4),
// column l%32 of its 32 x 32 tile.
#include "common.hpp"
#include "kentry.hpp"
#include "kernels.hpp"
#include "kmma.hpp"
#include "prof.hpp"

#include <algorithm>

namespace rr {

typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
constexpr int KS2_BM = 128, KS2_BN = 512, KS2_BK = 32;
constexpr int KS2_WC = 4;                              // 32-column MFMA tiles per wave
constexpr int KS2_WAVES = 2 * (KS2_BN / 32) / KS2_WC;  // two 64-row halves
constexpr int KS2_THREADS = 64 * KS2_WAVES;
constexpr int KS2_CPT = 4 * KS2_BN / KS2_THREADS;      // 16-byte Omega chunks per thread
constexpr int KS2_AS = 40;   // padded LDS row length (bf16) of the kernel tile
constexpr int KS2_BS = 40;   // padded LDS column length (bf16) of the Omega slice

struct Ks2Smem {
    uint16_t a_hi[2][KS2_BM * KS2_AS];
    uint16_t a_lo[2][KS2_BM * KS2_AS];
    uint16_t b[2][KS2_BN * KS2_BS];
};

// Omega slice of one step: thread t owns column c0 + t and its 32 points, as
// four 16-byte chunks (global loads into registers ahead of use; the LDS
// store of consecutive columns hits distinct banks).  B's rows [n, round8(n))
// are zero, so a chunk is either inside the padded column or wholly past it.
RR_DEV void ks2_load_b(const uint16_t* src, int64_t npad, int64_t k0, int cb, uint4 (&rb)[KS2_CPT]) {
#pragma unroll
    for (int s = 0; s < KS2_CPT; ++s) {
        const int64_t gj = k0 + 8 * (cb + s);
        rb[s] = (src && gj < npad) ? *(const uint4*)(src + gj) : make_uint4(0u, 0u, 0u, 0u);
    }
}
RR_DEV void ks2_store_b(Ks2Smem& sm, int buf, int col, int cb, const uint4 (&rb)[KS2_CPT]) {
#pragma unroll
    for (int s = 0; s < KS2_CPT; ++s) *(uint4*)&sm.b[buf][col * KS2_BS + 8 * (cb + s)] = rb[s];
}

// One step of MFMAs for the wave's 64 x (32 KS2_WC) tile, in two half steps of 16
// points; the second half step's operands are read from LDS while the first one's
// MFMAs run.
RR_DEV void ks2_mfma(const Ks2Smem& sm, int buf, int lane, int rh, int cq, f32x16_t (&acc)[2][KS2_WC]) {
    const int kq = 8 * (lane >> 5);
    bf16x8_t ah[2][2], al[2][2], bv[2][KS2_WC];
    auto load = [&](int kh) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row = rh * 64 + u * 32 + (lane & 31);
            ah[kh][u] = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sm.a_hi[buf][row * KS2_AS + 16 * kh + kq]);
            al[kh][u] = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sm.a_lo[buf][row * KS2_AS + 16 * kh + kq]);
        }
#pragma unroll
        for (int v = 0; v < KS2_WC; ++v) {
            const int col = cq * 32 * KS2_WC + v * 32 + (lane & 31);
            bv[kh][v] = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sm.b[buf][col * KS2_BS + 16 * kh + kq]);
        }
    };
    load(0);
    load(1);
#pragma unroll
    for (int kh = 0; kh < 2; ++kh)
#pragma unroll
        for (int v = 0; v < KS2_WC; ++v)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                acc[u][v] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kh][u], bv[kh][v], acc[u][v], 0, 0, 0);
                acc[u][v] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[kh][u], bv[kh][v], acc[u][v], 0, 0, 0);
            }
}

// SRHT Omega generated on the device (no Omega stream): Omega[i, c] =
// D_i (-1)^popcount(i & s_c) for i < n, zero past n.  For a step of 32 points
// starting at k (a multiple of 32), popcount((k + p) & s) = popcount(k & s) +
// popcount(p & s & 31), so the step's 32 signs of column c are one word:
// (parity(k & s_c) ? ~0 : 0) ^ W_c ^ (sign bits of D at k .. k+31), with W_c the
// column's 32-bit Walsh word.  Each byte of it indexes a 256-entry LDS table of
// 8 bf16 values +-1, written into the Omega slice in LDS as if it had been loaded.
RR_DEV void ks2_gen_slice(Ks2Smem& sm, int buf, int col, const uint4* table, uint64_t s, uint32_t w32,
                          int64_t k, uint32_t dw, int64_t n) {
    const uint32_t par = (uint32_t)__popcll((unsigned long long)((uint64_t)k & s)) & 1u;
    const uint32_t sg = (0u - par) ^ w32 ^ dw;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint4 v = table[(sg >> (8 * q)) & 0xFFu];
        const int64_t base = k + 8 * q;
        if (base + 8 > n) {   // last step only: zero the points past n
            const int64_t valid = n - base;
            uint32_t* w = &v.x;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t lo = (2 * j < valid) ? 0x0000FFFFu : 0u;
                const uint32_t hi = (2 * j + 1 < valid) ? 0xFFFF0000u : 0u;
                w[j] &= lo | hi;
            }
        }
        *(uint4*)&sm.b[buf][col * KS2_BS + 8 * q] = v;
    }
}

// part == nullptr: Y = scale * acc + mu * B.  Otherwise part[z] (n x m, leading
// dimension n) = acc over the block's point range [z*kper, (z+1)*kper).
// GEN: Omega is an SRHT given by its sampled rows srow (m) and the sign bits dbits
// of D (bit i%32 of word i/32), and its slices are generated instead of loaded.
template <int KIND, int DM, bool GEN>
__global__ __launch_bounds__(KS2_THREADS) void k_ksketch_bf16x2(
    int64_t n, const float* __restrict__ xa, const float* __restrict__ sqn, float c, float scale,
    float mu, const uint16_t* __restrict__ Bm, int64_t ldb, int64_t m, float* __restrict__ Y,
    int64_t ldy, int64_t kper, float* __restrict__ part, const int32_t* __restrict__ srow,
    const uint32_t* __restrict__ dbits) {
    constexpr int KB = KmmaShape<DM>::KB, NX = kmma_ncoord<DM>();
    // column-form records of the block's rows: in LDS, or for long records (which
    // would not fit beside the tiles) in the forming lanes' registers
    constexpr bool RREG = DM > 16;
    __shared__ __attribute__((aligned(16))) Ks2Smem sm;
    __shared__ uint4 gtable[GEN ? 256 : 1];
    __shared__ bf16x8_t rowrec[RREG ? 1 : KS2_BM * KB * 2];
    bf16x8_t rowreg[RREG ? KB : 1];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int rh = wave & 1, cq = wave >> 1;
    const bool former = wave < 4;   // forms kernel-tile rows 32*wave .. +31
    const int64_t i0 = (int64_t)blockIdx.x * KS2_BM;
    const int64_t c0 = (int64_t)blockIdx.y * KS2_BN;
    const int64_t kb = (int64_t)blockIdx.z * kper;
    const int64_t ke = (kb + kper < n) ? kb + kper : n;
    const float g = KIND == 1 ? c : 1.0f;

    // forming lanes: the record of row 32*wave + l32 into LDS, and the coordinates
    // of the step's point kb + l32 (rows and points past n: the last point; its
    // products meet zero rows of Omega or are not stored)
    const int frow = 32 * (wave & 3) + l32;
    float xr[NX], sqr = 0.0f;
    if (former) {
        const int64_t gi = i0 + frow;
        const int64_t gic = gi < n ? gi : n - 1;
        kmma_record<DM, false>(xa + gic * DM, sqn[gic], g, h, [&](int s, const bf16x8_t& v) {
            if constexpr (RREG) rowreg[s] = v;
            else rowrec[(frow * KB + s) * 2 + h] = v;
        });
        const int64_t gj = kb + l32 < n ? kb + l32 : n - 1;
        kmma_coords<DM>(xa + gj * DM, h, xr);
        sqr = sqn[gj];
    }
    // kernel tile of step k (points k .. k+31) into buffer b: the wave's 32 rows
    auto form = [&](int64_t k, int b) {
        f32x16_t d;
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = 0.0f;
        kmma_record_x<DM, true>(xr, sqr, g, h, [&](int s, const bf16x8_t& v) {
            const bf16x8_t rr = RREG ? rowreg[s] : rowrec[(frow * KB + s) * 2 + h];
            d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v, rr, d, 0, 0, 0);
        });
        // coordinates of the point one step further on
        const int64_t gj = k + KS2_BK + l32 < n ? k + KS2_BK + l32 : n - 1;
        kmma_coords<DM>(xa + gj * DM, h, xr);
        sqr = sqn[gj];
        // lane: row frow, points 8 g4 + 4 h + (0..3) of the step
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            bf16x4_t hv, lv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float kv = kmma_entry<KIND>(d[4 * g4 + r], c);
                const __bf16 hb = (__bf16)kv;
                hv[r] = hb;
                lv[r] = (__bf16)(kv - (float)hb);
            }
            *reinterpret_cast<bf16x4_t*>(&sm.a_hi[b][frow * KS2_AS + 8 * g4 + 4 * h]) = hv;
            *reinterpret_cast<bf16x4_t*>(&sm.a_lo[b][frow * KS2_AS + 8 * g4 + 4 * h]) = lv;
        }
    };

    f32x16_t acc[2][KS2_WC];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < KS2_WC; ++v)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[u][v][j] = 0.0f;

    // Omega staging: thread t owns chunks cb .. cb + KS2_CPT - 1 of column bcol
    const int bcol = t / (4 / KS2_CPT), bcb = (t % (4 / KS2_CPT)) * KS2_CPT;
    const uint16_t* bsrc = (c0 + bcol < m) ? Bm + (c0 + bcol) * ldb : nullptr;
    const int64_t npad = (n + 7) & ~(int64_t)7;   // B rows [n, npad) hold zeros
    if constexpr (GEN) {
        // sign table: entry e = the 8 bf16 values (-1 where bit t of e is set, else +1)
        if (t < 256) {
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                w[j] = (((uint32_t)t >> (2 * j)) & 1u ? 0xBF80u : 0x3F80u) |
                       ((((uint32_t)t >> (2 * j + 1)) & 1u ? 0xBF80u : 0x3F80u) << 16);
            gtable[t] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        // thread t generates column c0 + t of each slice (columns past m: zeros of no
        // consequence, their products are not stored)
        const int64_t gcol = c0 + t;
        const uint64_t scol = gcol < m ? (uint64_t)(uint32_t)srow[gcol] : 0ull;
        uint32_t w32 = 0;
#pragma unroll
        for (int p = 0; p < 32; ++p) w32 |= ((uint32_t)__popc((uint32_t)p & (uint32_t)scol) & 1u) << p;
        __syncthreads();   // row records, sign table
        if (kb < ke) {
            ks2_gen_slice(sm, 0, t, gtable, scol, w32, kb, dbits[kb >> 5], n);
            if (former) form(kb, 0);
        }
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = kb; k0 < ke; k0 += KS2_BK) {
            const int64_t k1 = k0 + KS2_BK;
            if (k1 < ke) {
                ks2_gen_slice(sm, buf ^ 1, t, gtable, scol, w32, k1, dbits[k1 >> 5], n);
                if (former) form(k1, buf ^ 1);
            }
            ks2_mfma(sm, buf, lane, rh, cq, acc);
            __syncthreads();
            buf ^= 1;
        }
    } else {
    // Omega slices in registers, two sets used by alternate steps: the slice that a
    // step stores into LDS was loaded two steps earlier (three steps before its
    // product MFMAs run), which covers the latency of these column-strided loads.
    // Loads past the block's point range stay inside B (rows past round8(n) read
    // as zeros).
    uint4 rx[KS2_CPT], ry[KS2_CPT];
    __syncthreads();   // row records
    if (kb < ke) {
        ks2_load_b(bsrc, npad, kb, bcb, rx);
        ks2_store_b(sm, 0, bcol, bcb, rx);
        if (former) form(kb, 0);
        ks2_load_b(bsrc, npad, kb + KS2_BK, bcb, rx);
        ks2_load_b(bsrc, npad, kb + 2 * KS2_BK, bcb, ry);
    }
    __syncthreads();
    int buf = 0;
    // one step at kc: rb holds slice kc + 32, refilled with slice kc + 96
    auto step = [&](int64_t kc, uint4 (&rb)[KS2_CPT]) {
        const int64_t k1 = kc + KS2_BK;
        if (k1 < ke) {
            ks2_store_b(sm, buf ^ 1, bcol, bcb, rb);
            ks2_load_b(bsrc, npad, kc + 3 * KS2_BK, bcb, rb);
        }
        // the forming wave of each SIMD builds the next tile while its partner's
        // product MFMAs run, then issues its own
        if (former && k1 < ke) form(k1, buf ^ 1);
        ks2_mfma(sm, buf, lane, rh, cq, acc);
        __syncthreads();
        buf ^= 1;
    };
    for (int64_t k0 = kb; k0 < ke; k0 += 2 * KS2_BK) {
        step(k0, rx);
        if (k0 + KS2_BK < ke) step(k0 + KS2_BK, ry);
    }
    }
    float* out = part ? part + (int64_t)blockIdx.z * ldy * m : Y;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int v = 0; v < KS2_WC; ++v) {
            const int64_t gc = c0 + cq * 32 * KS2_WC + v * 32 + (lane & 31);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t gr = i0 + rh * 64 + u * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
                if (gr < n && gc < m) {
                    if (part) {
                        out[gr + gc * ldy] = acc[u][v][j];
                    } else {
                        const float bval = __uint_as_float((uint32_t)Bm[gc * ldb + gr] << 16);
                        out[gr + gc * ldy] = fmaf(scale, acc[u][v][j], mu * bval);
                    }
                }
            }
        }
    }
}

// Y = scale * sum_z part[z] + mu * B, the splits added in order.
__global__ void k_ksketch_finish(int64_t n, int64_t m, int nsplit, const float* __restrict__ part,
                                 float scale, float mu, const uint16_t* __restrict__ Bm, int64_t ldb,
                                 float* __restrict__ Y, int64_t ldy) {
    const int64_t total = n * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        float s = 0.0f;
        for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * ldy * m + i + c * ldy];
        const float bval = __uint_as_float((uint32_t)Bm[c * ldb + i] << 16);
        Y[i + c * ldy] = fmaf(scale, s, mu * bval);
    }
}

// Number of point-range splits: fills whole rounds of the 256 compute units
// (one block each) as evenly as possible, at most 4.
static int ks2_splits(int64_t n, int64_t m) {
    const int64_t tiles = ((n + KS2_BM - 1) / KS2_BM) * ((m + KS2_BN - 1) / KS2_BN);
    const int64_t steps = (n + KS2_BK - 1) / KS2_BK;
    int best = 1;
    double best_eff = 0.0;
    for (int s = 1; s <= 4; ++s) {
        if (s > 1 && steps < 16 * s) break;
        const int64_t items = tiles * s;
        const int64_t rounds = (items + 255) / 256;
        const double eff = (double)items / (double)(rounds * 256);
        if (eff > best_eff + 0.03) { best_eff = eff; best = s; }
    }
    return best;
}

size_t kernel_sketch_ws_floats(int64_t n, int64_t m) {
    const int s = ks2_splits(n, m);
    return s > 1 ? (size_t)s * (size_t)n * (size_t)m : 0;
}

void launch_kernel_gemm_bf16x2(const KernelOp& op, const void* Bbf16, int64_t ldb, int64_t m,
                               double mu, float* Y, int64_t ldy, float* ws, hipStream_t st,
                               const int32_t* srht_rows, const uint32_t* srht_dbits) {
    const float c = kernel_c32(op.kind, op.kconst);
    const int ns = ks2_splits(op.n, m);
    const int64_t steps = (op.n + KS2_BK - 1) / KS2_BK;
    const int64_t kper = ((steps + ns - 1) / ns) * KS2_BK;
    float* part = ns > 1 ? ws : nullptr;
    dim3 grid((unsigned)((op.n + KS2_BM - 1) / KS2_BM), (unsigned)((m + KS2_BN - 1) / KS2_BN),
              (unsigned)ns);
    const uint16_t* B = (const uint16_t*)Bbf16;
    const float sc = (float)op.scale, fmu = (float)mu;
    ProfScope prof(PROF_KERNEL_SKETCH, st);
    const bool gen = srht_rows && srht_dbits;
#define KS2L(K, DD)                                                                                    \
    do {                                                                                               \
        if (gen)                                                                                       \
            k_ksketch_bf16x2<K, DD, true><<<grid, KS2_THREADS, 0, st>>>(op.n, op.xa, op.sqn, c, sc, fmu, B, \
                ldb, m, Y, ldy, kper, part, srht_rows, srht_dbits);                                    \
        else                                                                                           \
            k_ksketch_bf16x2<K, DD, false><<<grid, KS2_THREADS, 0, st>>>(op.n, op.xa, op.sqn, c, sc, fmu, B, \
                ldb, m, Y, ldy, kper, part, nullptr, nullptr);                                         \
    } while (0)
#define KS2D(K)                              \
    switch (op.dm) {                         \
        case 4: KS2L(K, 4); break;           \
        case 8: KS2L(K, 8); break;           \
        case 16: KS2L(K, 16); break;         \
        default: KS2L(K, 32); break;         \
    }
    if (op.kind == 1) { KS2D(1) } else { KS2D(2) }
#undef KS2D
#undef KS2L
    if (part) {
        int64_t g = (op.n * m + 255) / 256;
        if (g > 16384) g = 16384;
        k_ksketch_finish<<<(unsigned)g, 256, 0, st>>>(op.n, m, ns, part, sc, fmu, B, ldb, Y, ldy);
    }
}

}  // namespace rr
