// Reduced-precision hot path on the gfx950 matrix cores (MFMA).  Same
// persistent (channel, spectrum) schedule, decoding and FP32 gather gridding
// as the FP32 kernel; the two transform passes of Eq. 4 become dense products
// with the exp(+2 pi i ...) DFT matrix F (FP16 operands, FP32 accumulation):
//
//   row pass     Y   = G  F_W      [P*R rows x W]    x [W x N]     per spectrum
//   column pass  E~  = F_R Y        [N x R]           x [R x N]     per spectrum, pol
//
// each written in real form with the 2x2 block matrix M = [[Fr, -Fi], [Fi, Fr]]
// (so one real product gives both real and imaginary parts), K padded to
// whole 32-deep MFMA steps (zero cells beyond the aperture window, which sits
// at the grid origin as in the FP32 kernel).  G and Y are rounded to FP16 as
// MFMA inputs (4-bit samples times FP32 kernel weights); every accumulation,
// the polarisation products of Eq. 5 and the time sum stay in FP32.
//
// Wave w of a workgroup owns image rows 16w..16w+15 (j, m axis) and all of
// the workgroup's columns: its M fragments for those rows stay in registers
// for the whole kernel, and the X and Y outputs of each pixel land in the same
// lane and register slot, so the products and time sums never leave registers.
// MFMA 16x16x32 f16 lane layout (verified on the device): A lane l holds
// A[l%16][8(l/16)+e], B lane l holds B[8(l/16)+e][l%16], D lane l holds
// D[4(l/16)+e][l%16].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "epic_device.hpp"
#include "epic_gather.hpp"
#include "epic_internal.hpp"

namespace epic {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct MfmaArgs {
    const uint8_t* samples;   // [T][C][A][P]
    int64_t T;
    int C, A, S;
    const ChanInfo* chans;
    const CellDesc* cells_desc;
    const uint2* grp_ant;
    const float4* grp_w;
    const _Float16* dft;      // [2N][K2] real-form DFT matrix, row-major
    float* slots;             // [S][C][NPP][N][N]
    int WP;                   // pitch encoded in the gather program's cell offsets
    int M1max;                // rows of the row-pass operand (multiple of 16)
    uint32_t off_w, off_gant, off_desc, off_smp, off_A1, off_B2;
    int nibble_order;
    int grid_wg, wg_per_xcd;
};

template <int N_, int KK_>
struct MShape {
    static constexpr int N = N_;
    static constexpr int KK = KK_;                 // 32-deep MFMA steps per product
    static constexpr int KPAD = 16 * KK;           // window extent padded (cells)
    static constexpr int K2 = 2 * KPAD;            // real-form depth: [re | im]
    static constexpr int KS = (N > 64) ? 2 : 1;    // image columns split over KS workgroups
    static constexpr int NK = N / KS;              // columns per workgroup
    static constexpr int IT = NK / 16;             // 16-column tiles per workgroup
    static constexpr int WAVES = N / 16;           // one wave per 16 image rows
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int NT1 = 2 / KS;             // row-pass output tiles per wave
    static constexpr int A1P = K2 + 8;             // LDS pitches (halfs)
    static constexpr int B2P = K2 + 8;
};

template <int N_>
constexpr int mfma_threads() { return 64 * (N_ / 16); }

__device__ __forceinline__ floatx4 mfma16(half8 a, half8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

template <int N_, int KK_, int P, bool REAL, bool PROG_LDS>
__global__ void __launch_bounds__(mfma_threads<N_>()) mfma_kernel(MfmaArgs a) {
    using Sh = MShape<N_, KK_>;
    constexpr int N = Sh::N, KK = Sh::KK, KPAD = Sh::KPAD, K2 = Sh::K2, KS = Sh::KS, NK = Sh::NK;
    constexpr int IT = Sh::IT, THREADS = Sh::THREADS, NT1 = Sh::NT1, A1P = Sh::A1P, B2P = Sh::B2P;
    constexpr int NPP = (P == 2) ? 4 : 1;
    constexpr int GF4 = group_f4<P, REAL>();
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, l4 = lane >> 4;

    const int b = blockIdx.x;
    const int g = (b & 7) * a.wg_per_xcd + (b >> 3);
    if (g >= a.grid_wg) return;
    const int64_t T = a.T;
    const int64_t total = (int64_t)a.C * KS * T;
    const int64_t L = (total + a.grid_wg - 1) / a.grid_wg;
    const int64_t f0 = (int64_t)g * L;
    const int64_t f1 = (f0 + L < total) ? f0 + L : total;
    if (f0 >= f1) return;

    extern __shared__ __align__(16) unsigned char smem[];
    float4* s_w = reinterpret_cast<float4*>(smem + a.off_w);
    uint2* s_gant = reinterpret_cast<uint2*>(smem + a.off_gant);
    uint2* s_desc = reinterpret_cast<uint2*>(smem + a.off_desc);
    float2* s_smp0 = reinterpret_cast<float2*>(smem + a.off_smp);   // two sample buffers
    float2* s_smp1 = s_smp0 + a.A * P;
    _Float16* s_A1 = reinterpret_cast<_Float16*>(smem + a.off_A1);
    _Float16* s_B2 = reinterpret_cast<_Float16*>(smem + a.off_B2);

    // column-pass operand: rows 16w.. (real part) and N + 16w.. (imaginary part)
    half8 a2[2][KK];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ks = 0; ks < KK; ++ks)
            a2[h][ks] = *reinterpret_cast<const half8*>(a.dft + (size_t)(h * N + 16 * wave + l16) * K2 + 32 * ks +
                                                        8 * l4);

    const int AP = a.A * P;
    const bool words = ((AP & 3) == 0) && ((reinterpret_cast<uintptr_t>(a.samples) & 3) == 0);
    const int nwords = AP >> 2;

    constexpr int kPre = 1;   // sample words per thread loaded one spectrum ahead (more are loaded directly)
    uint32_t pre[kPre];
    auto prefetch = [&](int vv, int64_t tt) {
        const uint32_t* row4 =
            reinterpret_cast<const uint32_t*>(a.samples + ((int64_t)tt * a.C + vv / KS) * AP);
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int w = tid + k * THREADS;
            pre[k] = (w < nwords) ? row4[w] : 0u;
        }
    };

    // decode one (t, c) row of A*P bytes into dst: the prefetched words first,
    // any further words straight from memory
    auto decode = [&](float2* dst, int cc, int64_t tt) {
        if (words) {
#pragma unroll
            for (int k = 0; k < kPre; ++k) {
                const int w = tid + k * THREADS;
                if (w < nwords) {
                    const uint32_t x = pre[k];
                    dst[4 * w + 0] = unpack44(x & 0xFFu, a.nibble_order);
                    dst[4 * w + 1] = unpack44((x >> 8) & 0xFFu, a.nibble_order);
                    dst[4 * w + 2] = unpack44((x >> 16) & 0xFFu, a.nibble_order);
                    dst[4 * w + 3] = unpack44(x >> 24, a.nibble_order);
                }
            }
            const uint32_t* row4 = reinterpret_cast<const uint32_t*>(a.samples + ((int64_t)tt * a.C + cc) * AP);
            for (int w = tid + kPre * THREADS; w < nwords; w += THREADS) {
                const uint32_t x = row4[w];
                dst[4 * w + 0] = unpack44(x & 0xFFu, a.nibble_order);
                dst[4 * w + 1] = unpack44((x >> 8) & 0xFFu, a.nibble_order);
                dst[4 * w + 2] = unpack44((x >> 16) & 0xFFu, a.nibble_order);
                dst[4 * w + 3] = unpack44(x >> 24, a.nibble_order);
            }
        } else {
            const uint8_t* row = a.samples + ((int64_t)tt * a.C + cc) * AP;
            for (int k = tid; k < AP; k += THREADS) dst[k] = unpack44(row[k], a.nibble_order);
        }
    };

    int v = (int)(f0 / T);
    int64_t t = f0 - (int64_t)v * T;
    if (words) prefetch(v, t);
    for (int64_t f = f0; f < f1;) {
        // one channel segment: spectra t .. t+n-1 of virtual channel v
        const int64_t n = (f1 - f < T - t) ? f1 - f : T - t;
        const int c = v / KS;
        const int kpart = v - c * KS;
        const int slot = g - (int)(((int64_t)v * T) / L);
        const ChanInfo ci = a.chans[c];
        const int n_cell = ci.n_cell;
        const int R4 = (ci.R + 3) & ~3;
        const int M1 = P * R4;
        const CellDesc* g_desc = a.cells_desc + ci.cell_off;
        const uint2* g_gant = a.grp_ant + ci.grp_off;
        const float4* g_w = a.grp_w + (int64_t)ci.grp_off * GF4;
        half8 b1[NT1][KK];   // row-pass operand for this wave's output tiles
#pragma unroll
        for (int u = 0; u < NT1; ++u) {
            const int nloc = 16 * (wave * NT1 + u) + l16;          // own-column index in [0, 2 NK)
            const int row = (nloc < NK) ? kpart * NK + nloc : N + kpart * NK + (nloc - NK);
#pragma unroll
            for (int ks = 0; ks < KK; ++ks)
                b1[u][ks] = *reinterpret_cast<const half8*>(a.dft + (size_t)row * K2 + 32 * ks + 8 * l4);
        }
        __syncthreads();   // the previous segment is done with every LDS buffer
        if constexpr (PROG_LDS) {
            for (int k = tid; k < ci.n_grp * GF4; k += THREADS) s_w[k] = g_w[k];
            for (int k = tid; k < ci.n_grp; k += THREADS) s_gant[k] = g_gant[k];
            for (int k = tid; k < n_cell; k += THREADS) s_desc[k] = g_desc[k];
        }
        // zero both operand buffers: cells outside the window, rows beyond R
        // and the padding up to whole MFMA steps are never written again
        {
            uint4* z1 = reinterpret_cast<uint4*>(s_A1);
            for (int k = tid; k < a.M1max * A1P / 8; k += THREADS) z1[k] = make_uint4(0, 0, 0, 0);
            uint4* z2 = reinterpret_cast<uint4*>(s_B2);
            for (int k = tid; k < P * NK * B2P / 8; k += THREADS) z2[k] = make_uint4(0, 0, 0, 0);
        }
        float acc[IT][4][NPP];
#pragma unroll
        for (int it = 0; it < IT; ++it)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int k = 0; k < NPP; ++k) acc[it][e][k] = 0.f;

        // decode the segment's first spectrum (the rest are decoded one step
        // ahead, into the other sample buffer, while the current one is gridded)
        decode(s_smp0, c, t);
        if (words && f + 1 < f1) {
            if (t + 1 < T) prefetch(v, t + 1);
            else prefetch(v + 1, 0);
        }
        __syncthreads();

        for (int64_t i = 0; i < n; ++i) {
            const int64_t tt = t + i;
            float2* s_smp = (i & 1) ? s_smp1 : s_smp0;
            float2* s_nxt = (i & 1) ? s_smp0 : s_smp1;

            // 2. gather gridding (FP32), stored as the FP16 row-pass operand:
            //    row p*R4 + r, columns [Re G(r, 0..) | Im G(r, 0..)]
            for (int k = tid; k < n_cell; k += THREADS) {
                const uint2 d = PROG_LDS ? s_desc[k] : g_desc[k];
                const int off = (int)(d.x & 0xFFFFu);
                const int ng = (int)(d.x >> 16);
                float2 gx = make_float2(0.f, 0.f), gy = make_float2(0.f, 0.f);
                for (int j = 0; j < ng; ++j) {
                    const int gg = (int)d.y + j;
                    const uint2 ia = PROG_LDS ? s_gant[gg] : g_gant[gg];
                    const float4* w = PROG_LDS ? s_w + gg * GF4 : g_w + (int64_t)gg * GF4;
                    gather_group<P, REAL>(gx, gy, w, ia, s_smp);
                }
                const int r = off / a.WP, w = off - r * a.WP;
                _Float16* dst = s_A1 + r * A1P + w;
                dst[0] = (_Float16)gx.x;
                dst[KPAD] = (_Float16)gx.y;
                if constexpr (P == 2) {
                    dst[R4 * A1P] = (_Float16)gy.x;
                    dst[R4 * A1P + KPAD] = (_Float16)gy.y;
                }
            }
            // 1'. decode the next spectrum of this segment into the other buffer
            if (i + 1 < n) {
                decode(s_nxt, c, tt + 1);
                if (words && f + i + 2 < f1) {
                    if (tt + 2 < T) prefetch(v, tt + 2);
                    else prefetch(v + 1, 0);
                }
            }
            __syncthreads();

            // 3a. row pass: [M1 x K2] x [K2 x 2 NK] on the matrix cores; each wave
            //     takes NT1 output tiles and writes them, rounded to FP16, as the
            //     column-pass operand B2[p][i][Re Y(0..) | Im Y(0..)]
            for (int mt = 0; mt < (M1 + 15) / 16; ++mt) {
                half8 af[KK];
#pragma unroll
                for (int ks = 0; ks < KK; ++ks)
                    af[ks] = *reinterpret_cast<const half8*>(s_A1 + (16 * mt + l16) * A1P + 32 * ks + 8 * l4);
                const int m0 = 16 * mt + 4 * l4;
#pragma unroll
                for (int u = 0; u < NT1; ++u) {
                    floatx4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KK; ++ks) d = mfma16(af[ks], b1[u][ks], d);
                    if (m0 < M1) {
                        const int p = (P == 2 && m0 >= R4) ? 1 : 0;
                        const int r0 = m0 - p * R4;
                        const int nloc = 16 * (wave * NT1 + u) + l16;
                        const int part = nloc >= NK ? 1 : 0;
                        const int iloc = nloc - part * NK;
                        half4 hv;
                        hv[0] = (_Float16)d[0]; hv[1] = (_Float16)d[1]; hv[2] = (_Float16)d[2]; hv[3] = (_Float16)d[3];
                        *reinterpret_cast<half4*>(s_B2 + (p * NK + iloc) * B2P + part * KPAD + r0) = hv;
                    }
                }
            }
            __syncthreads();

            // 3b + 4. column pass: E~ rows 16w.. for every own column tile, both
            //         pols, then the products of Eq. 5 accumulated in registers
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                floatx4 er[P], ei[P];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    er[p] = floatx4{0.f, 0.f, 0.f, 0.f};
                    ei[p] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KK; ++ks) {
                        const half8 bf = *reinterpret_cast<const half8*>(s_B2 + (p * NK + 16 * it + l16) * B2P +
                                                                         32 * ks + 8 * l4);
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

        // add the segment's sums into its slot; bin -> pixel (+N/2 mod N)
        float* base = a.slots + ((int64_t)slot * a.C + c) * NPP * N * N;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int ii = kpart * NK + 16 * it + l16 + N / 2;
            if (ii >= N) ii -= N;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int j = 16 * wave + 4 * l4 + e + N / 2;
                if (j >= N) j -= N;
#pragma unroll
                for (int k = 0; k < NPP; ++k) base[((int64_t)k * N + j) * N + ii] += acc[it][e][k];
            }
        }
        f += n;
        ++v;
        t = 0;
    }
}

// ---- launch shapes -----------------------------------------------------------
struct Layout {
    uint32_t off_w, off_gant, off_desc, off_smp, off_A1, off_B2;
    size_t total;
    int M1max;
};

int ks_of(int N) { return N > 64 ? 2 : 1; }

Layout layout(const SubDev& d, bool prog_lds) {
    Layout L{};
    size_t b = 0;
    auto take = [&](size_t n) {
        b = (b + 15) & ~(size_t)15;
        size_t o = b;
        b += n;
        return (uint32_t)o;
    };
    const int gf4 = d.real_taps ? (d.P == 2 ? 2 : 1) : (d.P == 2 ? 4 : 2);
    const int K2 = 32 * d.KK;
    const int NK = d.N / ks_of(d.N);
    const int R4max = (d.Rmax + 3) & ~3;
    L.M1max = (d.P * R4max + 15) / 16 * 16;
    L.off_w = prog_lds ? take((size_t)d.Gmax * gf4 * 16) : 0;
    L.off_gant = prog_lds ? take((size_t)d.Gmax * 8) : 0;
    L.off_desc = prog_lds ? take((size_t)d.CellMax * 8) : 0;
    L.off_smp = take((size_t)2 * d.A * d.P * sizeof(float2));
    L.off_A1 = take((size_t)L.M1max * (K2 + 8) * 2);
    L.off_B2 = take((size_t)d.P * NK * (K2 + 8) * 2);
    L.total = (b + 15) & ~(size_t)15;
    return L;
}

using KernelFn = void (*)(MfmaArgs);

template <int N, int KK, int P>
KernelFn pick3(bool real, bool prog) {
    if (real) return prog ? mfma_kernel<N, KK, P, true, true> : mfma_kernel<N, KK, P, true, false>;
    return prog ? mfma_kernel<N, KK, P, false, true> : mfma_kernel<N, KK, P, false, false>;
}

template <int N, int KK>
KernelFn pick2(int P, bool real, bool prog) {
    return P == 2 ? pick3<N, KK, 2>(real, prog) : pick3<N, KK, 1>(real, prog);
}

// Grid sizes 32..128 (multiples of 16) with window depth KK*16 <= min(N, 64).
KernelFn select_kernel(int N, int KK, int P, bool real, bool prog) {
    switch (N * 8 + KK) {
#define EPIC_K(NN, KKK) case NN * 8 + KKK: return pick2<NN, KKK>(P, real, prog);
        EPIC_K(32, 1) EPIC_K(32, 2)
        EPIC_K(48, 1) EPIC_K(48, 2) EPIC_K(48, 3)
        EPIC_K(64, 1) EPIC_K(64, 2) EPIC_K(64, 3) EPIC_K(64, 4)
        EPIC_K(96, 1) EPIC_K(96, 2) EPIC_K(96, 3) EPIC_K(96, 4)
        EPIC_K(128, 1) EPIC_K(128, 2) EPIC_K(128, 3) EPIC_K(128, 4)
#undef EPIC_K
    }
    return nullptr;
}

constexpr size_t kLdsLimit = 160 * 1024;

// FP64 real-form DFT matrix M[2N][K2]: row n (i = n mod N), column k
// (w = k mod KPAD): [[cos, -sin], [sin, cos]] of 2 pi (w i mod N) / N, i.e.
// row block 0 gives the real part and row block 1 the imaginary part of
// sum_w exp(+2 pi i w i / N) z_w for z stacked as [Re z | Im z].
__global__ void dft_matrix_kernel(_Float16* __restrict__ m, int N, int KPAD) {
    const int K2 = 2 * KPAD;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * N * K2) return;
    const int n = idx / K2, k = idx - n * K2;
    const int i = n % N, w = k % KPAD;
    double s, c;
    sincospi(2.0 * (double)((int64_t)w * i % N) / (double)N, &s, &c);
    const bool imrow = n >= N, imcol = k >= KPAD;
    const double v = imrow ? (imcol ? c : s) : (imcol ? -s : c);
    m[idx] = (_Float16)v;
}

}  // namespace

hipError_t mfma_configure(SubDev& d, int device, int num_cu) {
    const int need = std::max(d.Rmax, d.Wmax);
    d.KK = (need + 15) / 16;
    if (d.N < 32 || d.N > 128 || d.N % 16 != 0 || d.N == 80 || d.N == 112) return hipErrorNotSupported;
    if (d.KK < 1 || 16 * d.KK > d.N || d.KK > 4) return hipErrorNotSupported;
    d.KS = ks_of(d.N);
    d.threads = 64 * (d.N / 16);
    const Layout with = layout(d, true);
    const Layout without = layout(d, false);
    const bool prog = with.total <= kLdsLimit / 2 || (with.total <= kLdsLimit && without.total > kLdsLimit / 2);
    const Layout& L = prog ? with : without;
    if (L.total > kLdsLimit) return hipErrorNotSupported;
    d.lds_bytes = L.total;
    d.prog_lds = prog ? 1 : 0;
    int occ = 2;
    if (device >= 0) {
        KernelFn fn = select_kernel(d.N, d.KK, d.P, d.real_taps != 0, prog);
        if (!fn) return hipErrorNotSupported;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
        if (e != hipSuccess) return e;
        int blocks = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(fn), d.threads,
                                                         L.total);
        if (e != hipSuccess) return e;
        occ = blocks > 0 ? blocks : 1;
    }
    d.grid_wg = ((num_cu * occ + 7) / 8) * 8;
    return hipSuccess;
}

hipError_t launch_dft_matrix(const SubDev& d, hipStream_t st) {
    const int n = 2 * d.N * 32 * d.KK;
    dft_matrix_kernel<<<dim3((n + 255) / 256), dim3(256), 0, st>>>(reinterpret_cast<_Float16*>(d.dft16), d.N,
                                                                   16 * d.KK);
    return hipGetLastError();
}

hipError_t launch_mfma(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st) {
    const bool prog = d.prog_lds != 0;
    const Layout L = layout(d, prog);
    MfmaArgs a{};
    a.samples = samples;
    a.T = n_time;
    a.C = d.C; a.A = d.A; a.S = d.S;
    a.chans = d.chans;
    a.cells_desc = d.cells_desc;
    a.grp_ant = reinterpret_cast<const uint2*>(d.grp_ant);
    a.grp_w = reinterpret_cast<const float4*>(d.grp_w);
    a.dft = reinterpret_cast<const _Float16*>(d.dft16);
    a.slots = d.slots;
    a.WP = d.WP;
    a.M1max = L.M1max;
    a.off_w = L.off_w; a.off_gant = L.off_gant; a.off_desc = L.off_desc;
    a.off_smp = L.off_smp; a.off_A1 = L.off_A1; a.off_B2 = L.off_B2;
    a.nibble_order = d.nibble_order;
    a.grid_wg = d.grid_wg;
    a.wg_per_xcd = (d.grid_wg + 7) / 8;
    KernelFn fn = select_kernel(d.N, d.KK, d.P, d.real_taps != 0, prog);
    if (!fn) return hipErrorNotSupported;
    hipLaunchKernelGGL(fn, dim3(8 * a.wg_per_xcd), dim3(d.threads), L.total, st, a);
    return hipGetLastError();
}

}  // namespace epic
