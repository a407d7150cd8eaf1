// Reduced-precision hot path on the gfx950 matrix cores (MFMA), gather
// gridding.  Same persistent (channel, spectrum) schedule and decoding as the
// FP32 kernel, and the same FP32 gather gridding; the two transform passes of
// Eq. 4 become dense products with the exp(+2 pi i ...) DFT matrix (FP16
// operands, FP32 accumulation) and the products of Eq. 5 are summed in FP32
// registers -- the shared building blocks are in epic_mfma.hpp.  G and Y are
// rounded to FP16 as MFMA inputs (4-bit samples times FP32 kernel weights);
// every accumulation, the polarisation products and the time sum stay in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "epic_device.hpp"
#include "epic_gather.hpp"
#include "epic_internal.hpp"
#include "epic_mfma.hpp"
#include "epic_sched.hpp"

namespace epic {

namespace {

// One sub-array as the segment function sees it.
struct SegCtx {
    const uint8_t* samples;   // [T][C][A][P]
    const ChanInfo* chans;
    const CellDesc* cells_desc;
    const uint2* grp_ant;
    const float4* grp_w;
    const _Float16* dft;      // [2N][K2] real-form DFT matrix, row-major
    float* slots;             // [S][C][NPP][N][N]
    int C, A;
    int WP;                   // pitch encoded in the gather program's cell offsets
    int M1max;                // rows of the row-pass operand (multiple of 16), per buffer
    int nibble_order, prog_lds;
    int fresh;                // 1: the slots hold zeros, store instead of add
};

// LDS carve-up shared by every segment a workgroup runs.
struct LdsMap {
    uint32_t off_w, off_gant, off_desc, off_smp, off_A1, off_B2;
    int smp_stride;           // samples (h2v) between the two sample buffers
};

struct MfmaArgs {
    SegCtx sc;
    LdsMap lm;
    int64_t T;
    int V;                    // virtual channels C * KS
    int grid_wg, wg_per_xcd;
};

// Gather gridding of every non-empty window cell (FP32 sums), stored as the
// FP16 row-pass operand: row p*prow + r, columns [Re G(r, 0..) | Im G(r, 0..)].
// The program pointers are all in LDS or all in global memory.
template <int P, int WM, int KPAD, int A1P, int TH, typename DescP, typename AntP, typename WP_>
__device__ __forceinline__ void gather_cells(DescP desc, AntP gant, WP_ wts, int n_cell,
                                             const h2v* __restrict__ smp, int WP, int prow, _Float16* s_A1) {
    constexpr int GF4 = group_f4<P, WM>();
    for (int k = threadIdx.x; k < n_cell; k += TH) {
        const uint2 d = desc[k];
        const int off = (int)(d.x & 0xFFFFu);
        const int ng = (int)(d.x >> 16);
        float2 gx = make_float2(0.f, 0.f), gy = make_float2(0.f, 0.f);
        for (int j = 0; j < ng; ++j) {
            const int gg = (int)d.y + j;
            gather_group<P, WM>(gx, gy, wts + (int64_t)gg * GF4, gant[gg], smp);
        }
        const int r = off / WP, w = off - r * WP;
        _Float16* dst = s_A1 + r * A1P + w;
        dst[0] = (_Float16)gx.x;
        dst[KPAD] = (_Float16)gx.y;
        if constexpr (P == 2) {
            dst[prow * A1P] = (_Float16)gy.x;
            dst[prow * A1P + KPAD] = (_Float16)gy.y;
        }
    }
}

// Process the spectra [k0, k1) of a sequence (index s*T + t) of one
// sub-array with TH threads; sequence channel s is virtual channel
// v = s * vstep + voff (channel v / KS, column part v % KS).  Waves beyond
// N/16 only help with the decoding, gathering and clearing.  The spectra's
// cost offsets are base + k*w in units where workgroup g's share is Lc
// (slot choice in slot_of).
template <int N_, int KK_, int P, int WM, int TH>
__device__ __forceinline__ void mfma_run(const SegCtx& sc, const LdsMap& lm, unsigned char* smem, int64_t T, int g,
                                         int64_t k0, int64_t k1, int64_t base, int64_t w_cost, int64_t Lc,
                                         int vstep, int voff) {
    using Sh = MShape<N_, KK_>;
    constexpr int N = Sh::N, KK = Sh::KK, KPAD = Sh::KPAD, K2 = Sh::K2, KS = Sh::KS, NK = Sh::NK;
    constexpr int IT = Sh::IT, NT1 = Sh::NT1, A1P = Sh::A1P, B2P = Sh::B2P, WAVES = Sh::WAVES;
    constexpr bool OWN = Sh::OWN;   // column-owner form (two A1 buffers, no B2)
    constexpr int NPP = (P == 2) ? 4 : 1;
    constexpr int GF4 = group_f4<P, WM>();
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, l4 = lane >> 4;
    const bool mwave = (TH == 64 * WAVES) || wave < WAVES;   // waves owning image rows
    const int mw = mwave ? wave : 0;
    const bool prog = sc.prog_lds != 0;

    float4* s_w = reinterpret_cast<float4*>(smem + lm.off_w);
    uint2* s_gant = reinterpret_cast<uint2*>(smem + lm.off_gant);
    uint2* s_desc = reinterpret_cast<uint2*>(smem + lm.off_desc);
    h2v* s_smp0 = reinterpret_cast<h2v*>(smem + lm.off_smp);   // two sample buffers (FP16, exact)
    h2v* s_smp1 = s_smp0 + lm.smp_stride;
    _Float16* s_A1 = reinterpret_cast<_Float16*>(smem + lm.off_A1);
    _Float16* s_B2 = reinterpret_cast<_Float16*>(smem + lm.off_B2);

    // column-pass operand: rows 16w.. (real part) and N + 16w.. (imaginary
    // part); in the column-owner form every row tile
    half8 a2[2][KK];
    half8 a2o[2][OWN ? Sh::RT : 1][KK];
    if constexpr (OWN) load_col_fragments_own<Sh>(a2o, sc.dft, l16, l4);
    else load_col_fragments<Sh>(a2, sc.dft, mw, l16, l4);
    const int a1_stride = OWN ? sc.M1max * A1P : 0;   // halfs between the two A1 buffers

    const int AP = sc.A * P;
    const bool words = ((AP & 3) == 0) && ((reinterpret_cast<uintptr_t>(sc.samples) & 3) == 0);
    const int nwords = AP >> 2;
    constexpr int kPre = 1;   // sample words per thread loaded one spectrum ahead (more are loaded directly)
    uint32_t pre[kPre];
    auto prefetch = [&](int vv, int64_t tt) {
        const uint32_t* row4 =
            reinterpret_cast<const uint32_t*>(sc.samples + ((int64_t)tt * sc.C + vv / KS) * AP);
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int w = tid + k * TH;
            pre[k] = (w < nwords) ? row4[w] : 0u;
        }
    };
    // decode one (t, c) row of A*P bytes into dst: the prefetched words first,
    // any further words straight from memory
    auto decode = [&](h2v* dst, int cc, int64_t tt) {
        if (words) {
#pragma unroll
            for (int k = 0; k < kPre; ++k) {
                const int w = tid + k * TH;
                if (w < nwords) {
                    const uint32_t x = pre[k];
                    dst[4 * w + 0] = unpack44_h(x & 0xFFu, sc.nibble_order);
                    dst[4 * w + 1] = unpack44_h((x >> 8) & 0xFFu, sc.nibble_order);
                    dst[4 * w + 2] = unpack44_h((x >> 16) & 0xFFu, sc.nibble_order);
                    dst[4 * w + 3] = unpack44_h(x >> 24, sc.nibble_order);
                }
            }
            const uint32_t* row4 = reinterpret_cast<const uint32_t*>(sc.samples + ((int64_t)tt * sc.C + cc) * AP);
            for (int w = tid + kPre * TH; w < nwords; w += TH) {
                const uint32_t x = row4[w];
                dst[4 * w + 0] = unpack44_h(x & 0xFFu, sc.nibble_order);
                dst[4 * w + 1] = unpack44_h((x >> 8) & 0xFFu, sc.nibble_order);
                dst[4 * w + 2] = unpack44_h((x >> 16) & 0xFFu, sc.nibble_order);
                dst[4 * w + 3] = unpack44_h(x >> 24, sc.nibble_order);
            }
        } else {
            const uint8_t* row = sc.samples + ((int64_t)tt * sc.C + cc) * AP;
            for (int k = tid; k < AP; k += TH) dst[k] = unpack44_h(row[k], sc.nibble_order);
        }
    };

    int s_ch = (int)(k0 / T);   // sequence channel
    int64_t t = k0 - (int64_t)s_ch * T;
    int v = s_ch * vstep + voff;
    if (words) prefetch(v, t);
    for (int64_t f = k0; f < k1;) {
        // one channel segment: spectra t .. t+n-1 of virtual channel v
        const int64_t n = (k1 - f < T - t) ? k1 - f : T - t;
        const int c = v / KS;
        const int kpart = v - c * KS;
        const int slot = slot_of(g, s_ch, t, T, base, w_cost, Lc);
        const ChanInfo ci = sc.chans[c];
        const int n_cell = ci.n_cell;
        const int R4 = (ci.R + 3) & ~3;
        const int M1 = P * R4;
        const CellDesc* g_desc = sc.cells_desc + ci.cell_off;
        const uint2* g_gant = sc.grp_ant + ci.grp_off;
        const float4* g_w = sc.grp_w + (int64_t)ci.grp_off * GF4;
        half8 b1[NT1][KK];   // row-pass operand for this wave's output tiles
        if constexpr (OWN) load_row_fragments_own<Sh>(b1, sc.dft, mw, l16, l4);
        else load_row_fragments<Sh>(b1, sc.dft, kpart, mw, l16, l4);
        __syncthreads();   // the previous segment is done with every LDS buffer
        if (prog) {
            for (int k = tid; k < ci.n_grp * GF4; k += TH) s_w[k] = g_w[k];
            for (int k = tid; k < ci.n_grp; k += TH) s_gant[k] = g_gant[k];
            for (int k = tid; k < n_cell; k += TH) s_desc[k] = g_desc[k];
        }
        // zero both operand buffers: cells outside the window, rows beyond R
        // and the padding up to whole MFMA steps are never written again
        {
            uint4* z1 = reinterpret_cast<uint4*>(s_A1);
            for (int k = tid; k < (OWN ? 2 : 1) * sc.M1max * A1P / 8; k += TH) z1[k] = make_uint4(0, 0, 0, 0);
            if constexpr (!OWN) {
                uint4* z2 = reinterpret_cast<uint4*>(s_B2);
                for (int k = tid; k < P * NK * B2P / 8; k += TH) z2[k] = make_uint4(0, 0, 0, 0);
            }
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
        if (words && f + 1 < k1) {
            if (t + 1 < T) prefetch(v, t + 1);
            else prefetch(v + vstep, 0);
        }
        __syncthreads();

        for (int64_t i = 0; i < n; ++i) {
            const int64_t tt = t + i;
            h2v* s_smp = (i & 1) ? s_smp1 : s_smp0;
            h2v* s_nxt = (i & 1) ? s_smp0 : s_smp1;

            // Wave priorities as in the FP32 kernel: the latency-bound gathering
            // and row pass ahead of the column pass of a CU's other workgroups.
            __builtin_amdgcn_s_setprio(2);
            // 2. gather gridding (FP32), stored as the FP16 row-pass operand:
            //    row p*prow + r, columns [Re G(r, 0..) | Im G(r, 0..)]; the
            //    column-owner form alternates two buffers and puts each pol
            //    at a whole number of tiles
            _Float16* a1 = s_A1 + (i & 1) * a1_stride;
            const int prow = OWN ? KPAD : R4;
            if (prog)
                gather_cells<P, WM, KPAD, A1P, TH>(s_desc, s_gant, s_w, n_cell, s_smp, sc.WP, prow, a1);
            else
                gather_cells<P, WM, KPAD, A1P, TH>(g_desc, g_gant, g_w, n_cell, s_smp, sc.WP, prow, a1);
            // 1'. decode the next spectrum of this segment into the other buffer
            if (i + 1 < n) {
                decode(s_nxt, c, tt + 1);
                if (words && f + i + 2 < k1) {
                    if (tt + 2 < T) prefetch(v, tt + 2);
                    else prefetch(v + vstep, 0);
                }
            }
            __syncthreads();

            if constexpr (OWN) {
                // 3 + 4. both passes in registers; the next spectrum's gather
                // writes the other A1 buffer, so one barrier per spectrum
                // orders everything (this buffer is rewritten only after the
                // next spectrum's barrier, which every wave reaches after this)
                __builtin_amdgcn_s_setprio(0);
                if (mwave) own_pass<Sh, P>(a1, b1, a2o, acc, ci.R, l16, l4);
            } else {
                __builtin_amdgcn_s_setprio(1);
                // 3a. row pass on the matrix cores -> column-pass operand B2
                if (mwave) row_pass<Sh, P>(s_A1, s_B2, b1, M1, R4, mw, l16, l4);
                __syncthreads();

                __builtin_amdgcn_s_setprio(0);
                // 3b + 4. column pass, both pols, products of Eq. 5 into registers
                if (mwave) col_pass<Sh, P>(s_B2, a2, acc, l16, l4);
            }
        }

        // add the segment's sums into its slot; bin -> pixel (+N/2 mod N)
        if constexpr (OWN) {
            if (mwave) flush_slot_own<Sh, P>(sc.slots, slot, sc.C, c, acc, mw, l16, l4, sc.fresh != 0);
        } else {
            if (mwave) flush_slot<Sh, P>(sc.slots, slot, sc.C, c, kpart, acc, mw, l16, l4, sc.fresh != 0);
        }
        f += n;
        ++s_ch;
        v += vstep;
        t = 0;
    }
}

// One sub-array: persistent, equal contiguous runs of the (channel, spectrum)
// sequence, XCD-aware (consecutive runs share an XCD's L2).
template <int N_, int KK_, int P, int WM>
__global__ void __launch_bounds__(mfma_threads<N_>())
__attribute__((amdgpu_waves_per_eu(MShape<N_, KK_>::WAVES_PER_EU))) mfma_kernel(MfmaArgs a) {
    const int b = blockIdx.x;
    const int g = (b & 7) * a.wg_per_xcd + (b >> 3);
    if (g >= a.grid_wg) return;
    constexpr int KS = MShape<N_, KK_>::KS;
    const PartSplit ps = part_split(g, a.grid_wg, KS);
    const int64_t total = (int64_t)(a.V / KS) * a.T;   // this column part's (channel, spectrum) sequence
    const int64_t L = (total + ps.Gp - 1) / ps.Gp;
    int64_t k0, k1;
    owned_range(ps.gp, L, 0, 1, total, &k0, &k1);
    if (k0 >= k1) return;
    extern __shared__ __align__(16) unsigned char smem[];
    mfma_run<N_, KK_, P, WM, mfma_threads<N_>()>(a.sc, a.lm, smem, a.T, ps.gp, k0, k1, 0, 1, L, KS, ps.kpart);
}

// ---- several sub-arrays in one persistent launch ---------------------------
// The spectra of all sub-arrays form one sequence in which a spectrum of
// sub-array s costs w_s units (a cost model, or times measured by the plan's
// autotuner); workgroup g takes every spectrum whose cost offset falls in
// [g L, (g+1) L), L = ceil(total / G), so uneven sub-arrays still give every
// workgroup the same work.  Each sub-array runs its own compiled shape.
constexpr int kBatchThreads = 384;   // 6 waves: one per 16 image rows up to N = 96

struct BatchArgs {
    const uint8_t* samples[kMaxSub];
    const BatchSub* subs;     // device table [n_sub]
    LdsMap lm;
    int n_sub;
    int64_t T;
    int grid_wg, wg_per_xcd;
    int fresh;                // 1: the slots hold zeros, store instead of add
};

// (N, KK) shapes a batched launch can run
#define EPIC_BATCH_SHAPES(F)                                                              \
    F(32, 1) F(32, 2) F(48, 1) F(48, 2) F(48, 3) F(64, 1) F(64, 2) F(64, 3) F(64, 4)      \
    F(96, 1) F(96, 2) F(96, 3) F(96, 4)

template <int P, int WM>
__global__ void __launch_bounds__(kBatchThreads) batch_kernel(BatchArgs a) {
    const int b = blockIdx.x;
    const int g = (b & 7) * a.wg_per_xcd + (b >> 3);
    if (g >= a.grid_wg) return;
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t total = 0;
    for (int s = 0; s < a.n_sub; ++s) total += (int64_t)a.subs[s].V * a.T * a.subs[s].weight;
    const int64_t Lc = (total + a.grid_wg - 1) / a.grid_wg;
    int64_t base = 0;
    for (int s = 0; s < a.n_sub; ++s) {
        const BatchSub& bs = a.subs[s];
        const int64_t items = (int64_t)bs.V * a.T;
        const int64_t w = bs.weight;
        int64_t k0, k1;
        owned_range(g, Lc, base, w, items, &k0, &k1);
        if (k0 < k1) {
            SegCtx sc;
            sc.samples = a.samples[s];
            sc.chans = bs.chans;
            sc.cells_desc = bs.cells_desc;
            sc.grp_ant = reinterpret_cast<const uint2*>(bs.grp_ant);
            sc.grp_w = reinterpret_cast<const float4*>(bs.grp_w);
            sc.dft = reinterpret_cast<const _Float16*>(bs.dft);
            sc.slots = bs.slots;
            sc.fresh = a.fresh;
            sc.C = bs.C; sc.A = bs.A; sc.WP = bs.WP; sc.M1max = bs.M1max;
            sc.nibble_order = bs.nibble_order; sc.prog_lds = bs.prog_lds;
            switch (bs.N * 8 + bs.KK) {
#define EPIC_RUN(NN, KKK)                                                                           \
    case NN * 8 + KKK:                                                                              \
        mfma_run<NN, KKK, P, WM, kBatchThreads>(sc, a.lm, smem, a.T, g, k0, k1, base, w, Lc, 1, 0); \
        break;
                EPIC_BATCH_SHAPES(EPIC_RUN)
#undef EPIC_RUN
            }
        }
        base += items * w;
    }
}

// ---- launch shapes -----------------------------------------------------------
struct Layout {
    LdsMap lm;
    size_t total;
    int M1max;
};

int ks_of(int N) { return N <= 64 ? 1 : (N <= 128 ? 2 : (N <= 192 ? 4 : 8)); }

size_t take_aligned(size_t& b, size_t n) {
    b = (b + 15) & ~(size_t)15;
    const size_t o = b;
    b += n;
    return o;
}

// rows of one row-pass operand buffer: pols at R4 (padded to whole tiles), or
// at whole tiles KPAD in the column-owner form
int m1max_of(const SubDev& d) {
    if (own_form(d.N, d.KK)) return d.P * 16 * d.KK;
    return (d.P * ((d.Rmax + 3) & ~3) + 15) / 16 * 16;
}

// LDS bytes of the row-pass operand (two buffers in the column-owner form)
// and of the column-pass operand (none there)
size_t a1_bytes(const SubDev& d) {
    return (size_t)(own_form(d.N, d.KK) ? 2 : 1) * m1max_of(d) * (32 * d.KK + kPadH) * 2;
}
size_t b2_bytes(const SubDev& d) {
    return own_form(d.N, d.KK) ? 0 : (size_t)d.P * (d.N / ks_of(d.N)) * (32 * d.KK + kPadH) * 2;
}

Layout layout(const SubDev& d, bool prog_lds) {
    Layout L{};
    size_t b = 0;
    const int gf4 = group_f4_of(d.P, d.wmode);
    L.M1max = m1max_of(d);
    L.lm.off_w = prog_lds ? (uint32_t)take_aligned(b, (size_t)d.Gmax * gf4 * 16) : 0;
    L.lm.off_gant = prog_lds ? (uint32_t)take_aligned(b, (size_t)d.Gmax * 8) : 0;
    L.lm.off_desc = prog_lds ? (uint32_t)take_aligned(b, (size_t)d.CellMax * 8) : 0;
    L.lm.off_smp = (uint32_t)take_aligned(b, (size_t)2 * d.A * d.P * 4);
    L.lm.smp_stride = d.A * d.P;
    L.lm.off_A1 = (uint32_t)take_aligned(b, a1_bytes(d));
    L.lm.off_B2 = (uint32_t)take_aligned(b, b2_bytes(d));
    L.total = (b + 15) & ~(size_t)15;
    return L;
}

using KernelFn = void (*)(MfmaArgs);

template <int N, int KK>
KernelFn pick2(int P, int wm) {
    if (P == 2) {
        if (wm == kWComplex) return mfma_kernel<N, KK, 2, kWComplex>;
        return wm == kWShared ? mfma_kernel<N, KK, 2, kWShared> : mfma_kernel<N, KK, 2, kWReal>;
    }
    return wm == kWComplex ? mfma_kernel<N, KK, 1, kWComplex> : mfma_kernel<N, KK, 1, kWReal>;
}

// Grid sizes 32..128 (multiples of 16, not 80 / 112), 192 and 256, with
// window depth KK*16 <= min(N, 64).
KernelFn select_kernel(int N, int KK, int P, int wm) {
    switch (N * 8 + KK) {
#define EPIC_K(NN, KKK) case NN * 8 + KKK: return pick2<NN, KKK>(P, wm);
        EPIC_K(32, 1) EPIC_K(32, 2)
        EPIC_K(48, 1) EPIC_K(48, 2) EPIC_K(48, 3)
        EPIC_K(64, 1) EPIC_K(64, 2) EPIC_K(64, 3) EPIC_K(64, 4)
        EPIC_K(96, 1) EPIC_K(96, 2) EPIC_K(96, 3) EPIC_K(96, 4)
        EPIC_K(128, 1) EPIC_K(128, 2) EPIC_K(128, 3) EPIC_K(128, 4)
        EPIC_K(192, 1) EPIC_K(192, 2) EPIC_K(192, 3) EPIC_K(192, 4)
        EPIC_K(256, 1) EPIC_K(256, 2) EPIC_K(256, 3) EPIC_K(256, 4)
#undef EPIC_K
    }
    return nullptr;
}

using BatchFn = void (*)(BatchArgs);

BatchFn select_batch(int P, int wm) {
    if (P == 2) {
        if (wm == kWComplex) return batch_kernel<2, kWComplex>;
        return wm == kWShared ? batch_kernel<2, kWShared> : batch_kernel<2, kWReal>;
    }
    return wm == kWComplex ? batch_kernel<1, kWComplex> : batch_kernel<1, kWReal>;
}

bool batch_shape_ok(int N, int KK) {
    switch (N * 8 + KK) {
#define EPIC_OK_CASE(NN, KKK) case NN * 8 + KKK: return true;
        EPIC_BATCH_SHAPES(EPIC_OK_CASE)
#undef EPIC_OK_CASE
    }
    return false;
}

constexpr size_t kLdsLimit = 160 * 1024;

bool prefer_prog(size_t with, size_t without) {
    return with <= kLdsLimit / 2 || (with <= kLdsLimit && without > kLdsLimit / 2);
}

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

hipError_t mfma_configure(SubDev& d, int device, int num_cu, int force_prog) {
    const int need = std::max(d.Rmax, d.Wmax);
    d.KK = (need + 15) / 16;
    const bool grid_ok = (d.N >= 32 && d.N <= 128 && d.N % 16 == 0 && d.N != 80 && d.N != 112) || d.N == 192 ||
                         d.N == 256;
    if (!grid_ok) return hipErrorNotSupported;
    if (d.KK < 1 || 16 * d.KK > d.N || d.KK > 4) return hipErrorNotSupported;
    d.KS = ks_of(d.N);
    d.threads = 64 * (d.N / 16);
    const Layout with = layout(d, true);
    const Layout without = layout(d, false);
    const bool prog = force_prog < 0 ? prefer_prog(with.total, without.total) : force_prog != 0;
    const Layout& L = prog ? with : without;
    if (L.total > kLdsLimit) return hipErrorNotSupported;
    d.lds_bytes = L.total;
    d.prog_lds = prog ? 1 : 0;
    int occ = 2;
    if (device >= 0) {
        KernelFn fn = select_kernel(d.N, d.KK, d.P, d.wmode);
        if (!fn) return hipErrorNotSupported;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
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
    const Layout L = layout(d, d.prog_lds != 0);
    MfmaArgs a{};
    a.sc.samples = samples;
    a.sc.chans = d.chans;
    a.sc.cells_desc = d.cells_desc;
    a.sc.grp_ant = reinterpret_cast<const uint2*>(d.grp_ant);
    a.sc.grp_w = reinterpret_cast<const float4*>(d.grp_w);
    a.sc.dft = reinterpret_cast<const _Float16*>(d.dft16);
    a.sc.slots = d.slots;
    a.sc.fresh = d.fresh;
    a.sc.C = d.C; a.sc.A = d.A; a.sc.WP = d.WP; a.sc.M1max = L.M1max;
    a.sc.nibble_order = d.nibble_order; a.sc.prog_lds = d.prog_lds;
    a.lm = L.lm;
    a.T = n_time;
    a.V = d.C * d.KS;
    a.grid_wg = d.grid_wg;
    a.wg_per_xcd = (d.grid_wg + 7) / 8;
    KernelFn fn = select_kernel(d.N, d.KK, d.P, d.wmode);
    if (!fn) return hipErrorNotSupported;
    hipLaunchKernelGGL(fn, dim3(8 * a.wg_per_xcd), dim3(d.threads), L.total, st, a);
    return hipGetLastError();
}

// Shared launch shape of a batched plan: the LDS layout holds the largest of
// every buffer over the sub-arrays; the gather programs live in LDS only if
// all of them fit.  Every sub-array must be an FP16 shape of the batch
// catalogue with the same pol count and tap kind.  Fills bd (not the device
// table, which the caller builds once slots and weights are known).
hipError_t batch_configure(SubDev* subs, int n_sub, BatchDev& bd, int device, int num_cu) {
    const int P = subs[0].P, wm = subs[0].wmode;
    size_t gw = 0, ga = 0, gd = 0, smp = 0, a1 = 0, b2 = 0;
    for (int s = 0; s < n_sub; ++s) {
        SubDev& d = subs[s];
        if (d.P != P || d.wmode != wm) return hipErrorNotSupported;
        d.KK = (std::max(d.Rmax, d.Wmax) + 15) / 16;
        if (!batch_shape_ok(d.N, d.KK)) return hipErrorNotSupported;
        d.KS = ks_of(d.N);
        const int gf4 = group_f4_of(P, wm);
        gw = std::max(gw, (size_t)d.Gmax * gf4 * 16);
        ga = std::max(ga, (size_t)d.Gmax * 8);
        gd = std::max(gd, (size_t)d.CellMax * 8);
        smp = std::max(smp, (size_t)d.A * d.P);
        a1 = std::max(a1, a1_bytes(d));
        b2 = std::max(b2, b2_bytes(d));
    }
    auto lay = [&](bool prog, LdsMap& lm) {
        size_t b = 0;
        lm.off_w = prog ? (uint32_t)take_aligned(b, gw) : 0;
        lm.off_gant = prog ? (uint32_t)take_aligned(b, ga) : 0;
        lm.off_desc = prog ? (uint32_t)take_aligned(b, gd) : 0;
        lm.off_smp = (uint32_t)take_aligned(b, 2 * smp * 4);
        lm.smp_stride = (int)smp;
        lm.off_A1 = (uint32_t)take_aligned(b, a1);
        lm.off_B2 = (uint32_t)take_aligned(b, b2);
        return (b + 15) & ~(size_t)15;
    };
    LdsMap lw{}, ln{};
    const size_t tw = lay(true, lw), tn = lay(false, ln);
    const bool prog = prefer_prog(tw, tn);
    const size_t total = prog ? tw : tn;
    if (total > kLdsLimit) return hipErrorNotSupported;
    const LdsMap& lm = prog ? lw : ln;
    bd.off[0] = lm.off_w; bd.off[1] = lm.off_gant; bd.off[2] = lm.off_desc;
    bd.off[3] = lm.off_smp; bd.off[4] = lm.off_A1; bd.off[5] = lm.off_B2;
    bd.smp_stride = lm.smp_stride;
    bd.lds_bytes = total;
    bd.prog_lds = prog ? 1 : 0;
    bd.P = P;
    bd.wmode = wm;
    bd.threads = kBatchThreads;
    bd.kkmax = 0;
    int occ = 1;
    if (device >= 0) {
        BatchFn fn = select_batch(P, wm);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
        if (e != hipSuccess) return e;
        int blocks = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(fn), kBatchThreads,
                                                         total);
        if (e != hipSuccess) return e;
        occ = blocks > 0 ? blocks : 1;
    }
    bd.grid_wg = ((num_cu * occ + 7) / 8) * 8;
    for (int s = 0; s < n_sub; ++s) {
        subs[s].threads = kBatchThreads;
        subs[s].lds_bytes = total;
        subs[s].prog_lds = bd.prog_lds;
        subs[s].grid_wg = bd.grid_wg;
    }
    return hipSuccess;
}

// The table entry of one sub-array of a batched plan (host side).
BatchSub batch_entry(const SubDev& d, int weight) {
    BatchSub b{};
    b.chans = d.chans;
    b.cells_desc = d.cells_desc;
    b.grp_ant = d.grp_ant;
    b.grp_w = d.grp_w;
    b.dft = reinterpret_cast<const uint16_t*>(d.dft16);
    b.slots = d.slots;
    b.C = d.C; b.A = d.A; b.V = d.C * d.KS;
    b.N = d.N; b.KK = d.KK; b.KS = d.KS; b.NK = d.N / d.KS; b.IT = b.NK / 16; b.WAVES = d.N / 16;
    b.NT1 = (2 * b.NK / 16 + b.WAVES - 1) / b.WAVES; b.WP = d.WP; b.M1max = m1max_of(d);
    b.nibble_order = d.nibble_order; b.S = d.S; b.weight = weight; b.prog_lds = d.prog_lds;
    return b;
}

hipError_t launch_batch(const BatchDev& bd, const uint8_t* const* samples, int n_sub, int64_t n_time,
                        hipStream_t st) {
    BatchArgs a{};
    for (int s = 0; s < n_sub; ++s) a.samples[s] = samples[s];
    a.subs = bd.table;
    a.n_sub = n_sub;
    a.T = n_time;
    a.grid_wg = bd.grid_wg;
    a.wg_per_xcd = (bd.grid_wg + 7) / 8;
    a.lm.off_w = bd.off[0]; a.lm.off_gant = bd.off[1]; a.lm.off_desc = bd.off[2];
    a.lm.off_smp = bd.off[3]; a.lm.off_A1 = bd.off[4]; a.lm.off_B2 = bd.off[5];
    a.lm.smp_stride = bd.smp_stride;
    a.fresh = bd.fresh;
    BatchFn fn = select_batch(bd.P, bd.wmode);
    hipLaunchKernelGGL(fn, dim3(8 * a.wg_per_xcd), dim3(kBatchThreads), bd.lds_bytes, st, a);
    return hipGetLastError();
}

}  // namespace epic
