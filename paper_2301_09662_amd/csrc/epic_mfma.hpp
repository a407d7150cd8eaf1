// Matrix-core (MFMA) building blocks shared by the two reduced-precision hot
// kernels: the gather-gridding kernel (kernels_mfma.hip) and the block-GEMM
// gridding kernel (kernels_bgemm.hip).  Both run the two transform passes of
// Eq. 4 as dense products with the exp(+2 pi i ...) DFT matrix F in real form
// M = [[Fr, -Fi], [Fi, Fr]] (FP16 operands, FP32 accumulation):
//
//   row pass     Y  = G F_W     [P*R rows x W]  x [W x N]   per spectrum
//   column pass  E~ = F_R Y     [N x R]         x [R x N]   per spectrum, pol
//
// and square / cross-multiply the sky fields (Eq. 5) into FP32 registers.
// Wave w owns image rows 16w..16w+15; its DFT fragments stay in registers and
// the X and Y outputs of each pixel land in the same lane and register slot.
// MFMA 16x16x32 f16 lane layout (verified on the device): A lane l holds
// A[l%16][8(l/16)+e], B lane l holds B[8(l/16)+e][l%16], D lane l holds
// D[4(l/16)+e][l%16].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "epic_device.hpp"

namespace epic {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Row padding (halfs) of the matrix-core operand buffers in LDS.
constexpr int kPadH = 8;

// Column-owner form: wave w owns image columns 16w..16w+15 for every image
// row; its row pass produces exactly the transformed rows of those columns,
// which stay in registers as the column pass's operand, so the row-pass result
// never goes through LDS and a spectrum needs one barrier instead of two.  It
// holds the column-pass operand of every image row in registers, which at
// N = 48 and 64 costs a resident workgroup per CU: measured on the 256-antenna
// station (N = 64) it ran 0.63 ms against 0.59-0.61 ms for the row-owner
// form, so it is used for N = 32 only (0.010 against 0.012 ms on the
// 16-antenna array).
constexpr bool own_form(int N, int KK) { return N <= 32 && (N / 16) * KK <= 8; }

template <int N_, int KK_>
struct MShape {
    static constexpr int N = N_;
    static constexpr int KK = KK_;                 // 32-deep MFMA steps per product
    static constexpr int KPAD = 16 * KK;           // window extent padded (cells)
    static constexpr int K2 = 2 * KPAD;            // real-form depth: [re | im]
    // image columns split over KS workgroups: a wave keeps its 16 image rows'
    // products of NK columns in registers, at most 64 columns, and 32 for the
    // 16-wave workgroups of N = 256 (whose 128-register budget holds no more)
    static constexpr int KS = (N <= 64) ? 1 : (N <= 128 ? 2 : (N <= 192 ? 4 : 8));
    static constexpr int NK = N / KS;              // columns per workgroup
    static constexpr int IT = NK / 16;             // 16-column tiles per workgroup
    static constexpr int WAVES = N / 16;           // one wave per 16 image rows
    static constexpr int TILES1 = 2 * NK / 16;     // row-pass output tiles: [Re | Im] of NK columns
    static constexpr int NT1 = (TILES1 + WAVES - 1) / WAVES;   // row-pass output tiles per wave
    // waves beyond TILES1 / NT1 (grids above 128) sit the row pass out
    static constexpr bool ALL_ROW_WAVES = TILES1 == WAVES * NT1;
    static constexpr bool OWN = own_form(N, KK);
    static constexpr int RT = N / 16;              // image row tiles (column-owner form)
    // register budget: three waves per SIMD (168 VGPRs) for the small shapes,
    // where the extra resident workgroup outweighs a few spills (measured:
    // station N = 64, KK = 2: 0.75 -> 0.64 ms); the compiler's choice otherwise
    static constexpr int WAVES_PER_EU = (N <= 64 && KK <= 2) ? 3 : 1;
    static constexpr int A1P = K2 + kPadH;         // LDS pitches (halfs)
    static constexpr int B2P = K2 + kPadH;
};

template <int N_>
constexpr int mfma_threads() { return 64 * (N_ / 16); }

__device__ __forceinline__ floatx4 mfma16(half8 a, half8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Column-pass operand of wave mw: DFT rows 16 mw.. (real part) and N + 16 mw..
// (imaginary part).
template <class Sh>
__device__ __forceinline__ void load_col_fragments(half8 (&a2)[2][Sh::KK], const _Float16* __restrict__ dft, int mw,
                                                   int l16, int l4) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ks = 0; ks < Sh::KK; ++ks)
            a2[h][ks] = *reinterpret_cast<const half8*>(dft + (size_t)(h * Sh::N + 16 * mw + l16) * Sh::K2 + 32 * ks +
                                                        8 * l4);
}

// Row-pass operand of wave mw for column part kpart: the DFT rows of the
// wave's NT1 output tiles.
template <class Sh>
__device__ __forceinline__ void load_row_fragments(half8 (&b1)[Sh::NT1][Sh::KK], const _Float16* __restrict__ dft,
                                                   int kpart, int mw, int l16, int l4) {
#pragma unroll
    for (int u = 0; u < Sh::NT1; ++u) {
        if (!Sh::ALL_ROW_WAVES && mw * Sh::NT1 + u >= Sh::TILES1) continue;
        const int nloc = 16 * (mw * Sh::NT1 + u) + l16;          // own-column index in [0, 2 NK)
        const int row = (nloc < Sh::NK) ? kpart * Sh::NK + nloc : Sh::N + kpart * Sh::NK + (nloc - Sh::NK);
#pragma unroll
        for (int ks = 0; ks < Sh::KK; ++ks)
            b1[u][ks] = *reinterpret_cast<const half8*>(dft + (size_t)row * Sh::K2 + 32 * ks + 8 * l4);
    }
}

// Row pass of one spectrum: [M1 x K2] x [K2 x 2 NK] on the matrix cores; each
// wave takes NT1 output tiles and writes them, rounded to FP16, as the
// column-pass operand B2[p][i][Re Y(0..) | Im Y(0..)].  s_A1 holds the
// spectrum's gridded window, row p*R4 + r: [Re G(r, 0..) | Im G(r, 0..)];
// rows beyond M1 (up to the next 16) may hold anything: their products are
// never stored.
template <class Sh, int P>
__device__ __forceinline__ void row_pass(const _Float16* __restrict__ s_A1, _Float16* __restrict__ s_B2,
                                         const half8 (&b1)[Sh::NT1][Sh::KK], int M1, int R4, int mw, int l16,
                                         int l4) {
    constexpr int KK = Sh::KK, NT1 = Sh::NT1, NK = Sh::NK, A1P = Sh::A1P, B2P = Sh::B2P, KPAD = Sh::KPAD;
    auto tile = [&](int mt) {
        half8 af[KK];
#pragma unroll
        for (int ks = 0; ks < KK; ++ks)
            af[ks] = *reinterpret_cast<const half8*>(s_A1 + (16 * mt + l16) * A1P + 32 * ks + 8 * l4);
        const int m0 = 16 * mt + 4 * l4;
#pragma unroll
        for (int u = 0; u < NT1; ++u) {
            if (!Sh::ALL_ROW_WAVES && mw * NT1 + u >= Sh::TILES1) continue;
            floatx4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KK; ++ks) d = mfma16(af[ks], b1[u][ks], d);
            if (m0 < M1) {
                const int p = (P == 2 && m0 >= R4) ? 1 : 0;
                const int r0 = m0 - p * R4;
                const int nloc = 16 * (mw * NT1 + u) + l16;
                const int part = nloc >= NK ? 1 : 0;
                const int iloc = nloc - part * NK;
                half4 hv;
                hv[0] = (_Float16)d[0]; hv[1] = (_Float16)d[1];
                hv[2] = (_Float16)d[2]; hv[3] = (_Float16)d[3];
                *reinterpret_cast<half4*>(s_B2 + (p * NK + iloc) * B2P + part * KPAD + r0) = hv;
            }
        }
    };
    if constexpr (KK <= 2) {
        // at most four tiles: unrolled with a uniform exit, so every tile's
        // operand loads issue ahead of the products (station FP16 -4 %)
#pragma unroll
        for (int mt = 0; mt < (KPAD * P + 15) / 16; ++mt) {
            if (16 * mt >= M1) break;
            tile(mt);
        }
    } else {
        for (int mt = 0; mt < (M1 + 15) / 16; ++mt) tile(mt);
    }
}

// Column pass of one spectrum for wave mw's 16 image rows and every own
// column tile, both pols, then the products of Eq. 5 added into registers:
// acc[it][e][k], k = XX*, YY*, Re XY*, Im XY* (single pol: XX*).
template <class Sh, int P>
__device__ __forceinline__ void col_pass(const _Float16* __restrict__ s_B2, const half8 (&a2)[2][Sh::KK],
                                         float (&acc)[Sh::IT][4][(P == 2) ? 4 : 1], int l16, int l4) {
    constexpr int KK = Sh::KK, NK = Sh::NK, B2P = Sh::B2P;
#pragma unroll
    for (int it = 0; it < Sh::IT; ++it) {
        floatx4 er[P], ei[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            er[p] = floatx4{0.f, 0.f, 0.f, 0.f};
            ei[p] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KK; ++ks) {
                const half8 bf =
                    *reinterpret_cast<const half8*>(s_B2 + (p * NK + 16 * it + l16) * B2P + 32 * ks + 8 * l4);
                er[p] = mfma16(a2[0][ks], bf, er[p]);
                ei[p] = mfma16(a2[1][ks], bf, ei[p]);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float xr = er[0][e], xi = ei[0][e];
            acc[it][e][0] = fmaf(xr, xr, fmaf(xi, xi, acc[it][e][0]));
            if constexpr (P == 2) {
                const float yr = er[1][e], yi = ei[1][e];
                acc[it][e][1] = fmaf(yr, yr, fmaf(yi, yi, acc[it][e][1]));
                acc[it][e][2] = fmaf(xr, yr, fmaf(xi, yi, acc[it][e][2]));
                acc[it][e][3] = fmaf(xi, yr, fmaf(-xr, yi, acc[it][e][3]));
            }
        }
    }
}

// ---- column-owner form -------------------------------------------------------
// Column-pass operand of the column-owner form: every image row tile rt, real
// (h = 0) and imaginary (h = 1) output rows.  The depth is permuted to match
// the registers the row pass leaves: slot e of lane quarter l4 in 32-deep step
// ks is depth 16 (2 ks + e / 4) + 4 l4 + e % 4.
template <class Sh>
__device__ __forceinline__ void load_col_fragments_own(half8 (&a2)[2][Sh::RT][Sh::KK],
                                                       const _Float16* __restrict__ dft, int l16, int l4) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int rt = 0; rt < Sh::RT; ++rt)
#pragma unroll
            for (int ks = 0; ks < Sh::KK; ++ks) {
                const _Float16* row = dft + (size_t)(h * Sh::N + 16 * rt + l16) * Sh::K2 + 32 * ks + 4 * l4;
                const half4 lo = *reinterpret_cast<const half4*>(row);
                const half4 hi = *reinterpret_cast<const half4*>(row + 16);
                a2[h][rt][ks] = half8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            }
}

// Row-pass operand of wave w in the column-owner form: the DFT rows of its
// real (u = 0) and imaginary (u = 1) output columns 16w + l16.
template <class Sh>
__device__ __forceinline__ void load_row_fragments_own(half8 (&b1)[2][Sh::KK], const _Float16* __restrict__ dft,
                                                       int w, int l16, int l4) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int ks = 0; ks < Sh::KK; ++ks)
            b1[u][ks] = *reinterpret_cast<const half8*>(dft + (size_t)(u * Sh::N + 16 * w + l16) * Sh::K2 + 32 * ks +
                                                        8 * l4);
}

// Row pass and column pass of one spectrum in the column-owner form.  s_A1
// holds the gridded window with pol p's rows at p * KPAD + r (rows r >= R are
// zero).  For each pol the row pass yields the 2 KK 16-row tiles of the
// wave's transformed columns -- tile j: real part (j < KK) or imaginary part
// of rows 16 (j mod KK) .. -- which, rounded to FP16 and paired (2 ks, 2 ks + 1),
// are the column pass's depth steps ks; then the products of Eq. 5 are added
// into acc[rt][e][k] for image row 16 rt + 4 l4 + e, image column 16 w + l16.
template <class Sh, int P>
__device__ __forceinline__ void own_pass(const _Float16* __restrict__ s_A1, const half8 (&b1)[2][Sh::KK],
                                         const half8 (&a2)[2][Sh::RT][Sh::KK],
                                         float (&acc)[Sh::RT][4][(P == 2) ? 4 : 1], int R, int l16, int l4) {
    constexpr int KK = Sh::KK, KPAD = Sh::KPAD, A1P = Sh::A1P;
    half8 yb[P][KK];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        floatx4 dt[2 * KK];
#pragma unroll
        for (int mt = 0; mt < KK; ++mt) {
            dt[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
            dt[KK + mt] = floatx4{0.f, 0.f, 0.f, 0.f};
            if (16 * mt < R) {   // uniform: tiles past the window rows are zero
                half8 af[KK];
#pragma unroll
                for (int ks = 0; ks < KK; ++ks)
                    af[ks] = *reinterpret_cast<const half8*>(s_A1 + (p * KPAD + 16 * mt + l16) * A1P + 32 * ks + 8 * l4);
#pragma unroll
                for (int ks = 0; ks < KK; ++ks) {
                    dt[mt] = mfma16(af[ks], b1[0][ks], dt[mt]);
                    dt[KK + mt] = mfma16(af[ks], b1[1][ks], dt[KK + mt]);
                }
            }
        }
#pragma unroll
        for (int ks = 0; ks < KK; ++ks) {
            const floatx4 a = dt[2 * ks], b = dt[2 * ks + 1];
            yb[p][ks] = half8{(_Float16)a[0], (_Float16)a[1], (_Float16)a[2], (_Float16)a[3],
                              (_Float16)b[0], (_Float16)b[1], (_Float16)b[2], (_Float16)b[3]};
        }
    }
#pragma unroll
    for (int rt = 0; rt < Sh::RT; ++rt) {
        floatx4 er[P], ei[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            er[p] = floatx4{0.f, 0.f, 0.f, 0.f};
            ei[p] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KK; ++ks) {
                er[p] = mfma16(a2[0][rt][ks], yb[p][ks], er[p]);
                ei[p] = mfma16(a2[1][rt][ks], yb[p][ks], ei[p]);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float xr = er[0][e], xi = ei[0][e];
            acc[rt][e][0] = fmaf(xr, xr, fmaf(xi, xi, acc[rt][e][0]));
            if constexpr (P == 2) {
                const float yr = er[1][e], yi = ei[1][e];
                acc[rt][e][1] = fmaf(yr, yr, fmaf(yi, yi, acc[rt][e][1]));
                acc[rt][e][2] = fmaf(xr, yr, fmaf(xi, yi, acc[rt][e][2]));
                acc[rt][e][3] = fmaf(xi, yr, fmaf(-xr, yi, acc[rt][e][3]));
            }
        }
    }
}

// Segment flush of the column-owner form (wave w: image columns 16w..).
template <class Sh, int P>
__device__ __forceinline__ void flush_slot_own(float* __restrict__ slots, int slot, int C, int c,
                                               const float (&acc)[Sh::RT][4][(P == 2) ? 4 : 1], int w, int l16,
                                               int l4, bool fresh) {
    constexpr int N = Sh::N, NPP = (P == 2) ? 4 : 1;
    float* base_p = slots + ((int64_t)slot * C + c) * NPP * N * N;
    int ii = 16 * w + l16 + N / 2;
    if (ii >= N) ii -= N;
#pragma unroll
    for (int rt = 0; rt < Sh::RT; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int j = 16 * rt + 4 * l4 + e + N / 2;
            if (j >= N) j -= N;
#pragma unroll
            for (int k = 0; k < NPP; ++k) slot_put(&base_p[((int64_t)k * N + j) * N + ii], acc[rt][e][k], fresh);
        }
}

// Add a segment's sums into its slot of channel c; frequency bin -> pixel
// (+N/2 mod N on both axes).
template <class Sh, int P>
__device__ __forceinline__ void flush_slot(float* __restrict__ slots, int slot, int C, int c, int kpart,
                                           const float (&acc)[Sh::IT][4][(P == 2) ? 4 : 1], int mw, int l16,
                                           int l4, bool fresh) {
    constexpr int N = Sh::N, NPP = (P == 2) ? 4 : 1;
    float* base_p = slots + ((int64_t)slot * C + c) * NPP * N * N;
#pragma unroll
    for (int it = 0; it < Sh::IT; ++it) {
        int ii = kpart * Sh::NK + 16 * it + l16 + N / 2;
        if (ii >= N) ii -= N;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int j = 16 * mw + 4 * l4 + e + N / 2;
            if (j >= N) j -= N;
#pragma unroll
            for (int k = 0; k < NPP; ++k) slot_put(&base_p[((int64_t)k * N + j) * N + ii], acc[it][e][k], fresh);
        }
    }
}

}  // namespace epic
