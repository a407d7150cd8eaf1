// Gridding on the matrix cores (EPIC_GRID_BLOCK_GEMM / EPIC_GRID_DENSE_GEMM).
//
// Gridding (Eq. 4: the antenna fields W_a * E_a summed over antennas) of a
// channel is the product G = Wc E of the channel's kernel matrix Wc [cells x
// antennas] with the spectra's fields E [antennas x (spectrum, pol, re/im)].
// With real weights one real product gives both the real and the imaginary
// part of every pol.  The product runs on 16 x 16 x 32 MFMA tiles:
//   rows     16 aperture cells of the channel's window (its non-empty cells
//            in raster order, 16 per tile);
//   depth    32 antennas, taken in raster order of their positions so that a
//            block of 32 touches only a few rows of cells;
//   columns  TB spectra x P pols x (re, im) of the current step.
// Only the (cell tile, antenna block) pairs that hold a non-zero weight are
// stored and multiplied (block-sparse form); the dense form keeps every
// antenna block of every tile.  The weights are split into parts in the
// operand type whose products are summed in FP32: FP16 high + low (~2^-22
// relative), or FP8 e4m3 with a power-of-two scale, high + middle + low, each
// part holding the previous one's rounding error times 16 (<= 2^-12 relative;
// two e4m3 parts leave up to 2^-8, which measurably exceeds the 1e-3 image bar
// for arrays of a few antennas).  The 4-bit samples are exact in either type.
// The gridded cells go
// to the FP16 row-pass operand, and the two transform passes, the products of
// Eq. 5 and the time sums run as in the gather-gridding kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "epic_device.hpp"
#include "epic_gather.hpp"
#include "epic_internal.hpp"
#include "epic_mfma.hpp"
#include "epic_sched.hpp"

namespace epic {

namespace {

// Operand of one 16 x 32 (A) or 32 x 16 (B) block per lane: 8 elements.
template <int OP>
struct Operand;
template <>
struct Operand<kBgFp16> {
    using type = half8;               // 16 bytes
    static constexpr int bytes = 2;
};
template <>
struct Operand<kBgFp8> {
    using type = long;                // 8 bytes of e4m3
    static constexpr int bytes = 1;
};

template <int OP>
__device__ __forceinline__ floatx4 mfma_op(typename Operand<OP>::type a, typename Operand<OP>::type b, floatx4 c) {
    if constexpr (OP == kBgFp16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// One element of the field operand: a 4-bit integer, exact in both types.
template <int OP>
__device__ __forceinline__ void put_elem(unsigned char* base, int idx, float v) {
    if constexpr (OP == kBgFp16) {
        reinterpret_cast<_Float16*>(base)[idx] = (_Float16)v;
    } else {
        base[idx] = (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xFF);
    }
}

struct BgArgs {
    const uint8_t* samples;   // [T][C][A][P]
    const ChanInfo* chans;
    const BgChan* bg;
    const uint2* tiles;       // (first block entry of the tile, channel-relative; block count)
    const uint16_t* cells;    // [tile][16] (r << 8 | w), 0xFFFF padding
    const uint16_t* ents;     // antenna block of each block entry
    const int32_t* perm;      // [A] antenna at raster position s
    const unsigned char* w;   // [term][entry][64 lanes][8] operand elements
    int64_t wterm;            // bytes between terms
    const float* scale;       // [2]: weight scale, its inverse
    const _Float16* dft;      // [2N][K2] real-form DFT matrix
    float* slots;             // [S][C][NPP][N][N]
    int fresh;                // 1: the slots hold zeros, store instead of add
    int64_t T;
    int C, A, nibble_order, TB, nablk, V;
    uint32_t off_E, off_A1, off_B2;
    int A1rows;               // rows of the A1 region (zeroed per segment)
    int grid_wg, wg_per_xcd;
};

// Register budget: two waves per SIMD for the grids up to 64 with at most two
// MFMA steps (their ~220 live registers fit without spilling: measured at the
// station shape, 1.19 ms with three waves and ~60 spilled registers against
// 0.80 ms with two); the compiler's choice otherwise.
template <int N_, int KK_>
constexpr int bg_waves_per_eu() { return (N_ <= 64 && KK_ <= 2) ? 2 : 1; }

template <int N_, int KK_, int P, int OP>
__global__ void __launch_bounds__(mfma_threads<N_>())
__attribute__((amdgpu_waves_per_eu(bg_waves_per_eu<N_, KK_>()))) bg_kernel(BgArgs a) {
    using Sh = MShape<N_, KK_>;
    using Op = typename Operand<OP>::type;
    constexpr int TH = mfma_threads<N_>(), NW = TH / 64;
    constexpr int KS = Sh::KS, KPAD = Sh::KPAD, A1P = Sh::A1P, B2P = Sh::B2P, NK = Sh::NK, IT = Sh::IT;
    constexpr int NPP = (P == 2) ? 4 : 1;
    constexpr int EB = Operand<OP>::bytes;
    constexpr int NTERM = (OP == kBgFp16) ? 2 : 3;
    const int b = blockIdx.x;
    const int g = (b & 7) * a.wg_per_xcd + (b >> 3);
    if (g >= a.grid_wg) return;
    const PartSplit ps = part_split(g, a.grid_wg, KS);
    const int64_t T = a.T;
    const int64_t total = (int64_t)(a.V / KS) * T;   // this column part's (channel, spectrum) sequence
    const int64_t L = (total + ps.Gp - 1) / ps.Gp;
    int64_t k0, k1;
    owned_range(ps.gp, L, 0, 1, total, &k0, &k1);
    if (k0 >= k1) return;

    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* s_E = smem + a.off_E;                                      // [nablk][64][8]
    _Float16* s_A1 = reinterpret_cast<_Float16*>(smem + a.off_A1);
    _Float16* s_B2 = reinterpret_cast<_Float16*>(smem + a.off_B2);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, l4 = lane >> 4;
    const int mw = wave;   // every wave owns 16 image rows
    const int kpart = ps.kpart;

    // the field operand rows of antennas beyond A (last block) stay zero
    {
        uint4* z = reinterpret_cast<uint4*>(s_E);
        for (int k = tid; k < a.nablk * 64 * 8 * EB / 16; k += TH) z[k] = make_uint4(0, 0, 0, 0);
    }
    half8 a2[2][Sh::KK];
    load_col_fragments<Sh>(a2, a.dft, mw, l16, l4);
    float inv_scale = 1.0f;
    if constexpr (OP == kBgFp8) inv_scale = a.scale[1];

    // decode spectra t .. t+nb-1 of channel c into the field operand: element
    // (antenna s, column n = u 2P + 2p + ri) of block s / 32 sits at lane
    // 16 ((s % 32) / 8) + n, position s % 8
    const int AP = a.A * P;
    auto decode = [&](int cc, int64_t t, int nb) {
        for (int task = tid; task < nb * a.A; task += TH) {
            const int u = task / a.A;
            const int s = task - u * a.A;
            const int an = a.perm[s];
            const uint8_t* row = a.samples + ((t + u) * a.C + cc) * (int64_t)AP + (int64_t)an * P;
            const int j = s >> 5, k = s & 31;
            const int base = (j * 64 + 16 * (k >> 3)) * 8 + (k & 7);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float2 v = unpack44(row[p], a.nibble_order);
                const int n = u * 2 * P + 2 * p;
                put_elem<OP>(s_E, base + n * 8, v.x);
                put_elem<OP>(s_E, base + (n + 1) * 8, v.y);
            }
        }
    };

    int s_ch = (int)(k0 / T);
    int64_t t = k0 - (int64_t)s_ch * T;
    int v = s_ch * KS + kpart;
    for (int64_t f = k0; f < k1;) {
        const int64_t n = (k1 - f < T - t) ? k1 - f : T - t;
        const int c = v / KS;
        const int slot = slot_of(ps.gp, s_ch, t, T, 0, 1, L);
        const ChanInfo ci = a.chans[c];
        const BgChan bc = a.bg[c];
        const int R4 = (ci.R + 3) & ~3;
        const int M1 = P * R4;
        __syncthreads();   // the previous segment is done with every LDS buffer
        {
            uint4* z1 = reinterpret_cast<uint4*>(s_A1);
            for (int k = tid; k < a.A1rows * A1P / 8; k += TH) z1[k] = make_uint4(0, 0, 0, 0);
            uint4* z2 = reinterpret_cast<uint4*>(s_B2);
            for (int k = tid; k < P * NK * B2P / 8; k += TH) z2[k] = make_uint4(0, 0, 0, 0);
        }
        float acc[IT][4][NPP];
#pragma unroll
        for (int it = 0; it < IT; ++it)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int k = 0; k < NPP; ++k) acc[it][e][k] = 0.f;

        decode(c, t, (int)std::min<int64_t>(a.TB, n));
        __syncthreads();

        for (int64_t u0 = 0; u0 < n; u0 += a.TB) {
            const int nb = (int)std::min<int64_t>(a.TB, n - u0);
            __builtin_amdgcn_s_setprio(2);
            // 2. gridding product: G rows (cells) x columns (u, p, re/im), two
            //    tiles of the wave at a time with the operands of two block
            //    entries of each in flight, so that the weight loads from L2
            //    overlap instead of queueing behind each other
            for (int i0 = wave; i0 < bc.n_tile; i0 += 2 * NW) {
                const int i1 = i0 + NW;
                const uint2 t0 = a.tiles[bc.tile_off + i0];
                const uint2 t1 = (i1 < bc.n_tile) ? a.tiles[bc.tile_off + i1] : make_uint2(0u, 0u);
                const int n0 = (int)t0.y, n1 = (int)t1.y;
                floatx4 d0[NTERM], d1[NTERM];
#pragma unroll
                for (int h = 0; h < NTERM; ++h) {
                    d0[h] = floatx4{0.f, 0.f, 0.f, 0.f};
                    d1[h] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
                auto load = [&](int ent, Op (&w)[NTERM], Op& eb) {
                    const unsigned char* src = a.w + ((size_t)ent * 64 + lane) * 8 * EB;
#pragma unroll
                    for (int h = 0; h < NTERM; ++h) w[h] = *reinterpret_cast<const Op*>(src + h * a.wterm);
                    eb = *reinterpret_cast<const Op*>(s_E + ((int)a.ents[ent] * 64 + lane) * 8 * EB);
                };
                const int nmax = n0 > n1 ? n0 : n1;
                for (int q0 = 0; q0 < nmax; q0 += 2) {
                    Op w0[2][NTERM], e0[2], w1[2][NTERM], e1[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        if (q0 + q < n0) load(bc.ent_off + (int)t0.x + q0 + q, w0[q], e0[q]);
                        if (q0 + q < n1) load(bc.ent_off + (int)t1.x + q0 + q, w1[q], e1[q]);
                    }
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        if (q0 + q < n0) {
                            if constexpr (OP == kBgFp16) {
                                d0[0] = mfma_op<OP>(w0[q][0], e0[q], d0[0]);
                                d0[0] = mfma_op<OP>(w0[q][1], e0[q], d0[0]);
                            } else {
#pragma unroll
                                for (int h = 0; h < NTERM; ++h) d0[h] = mfma_op<OP>(w0[q][h], e0[q], d0[h]);
                            }
                        }
                        if (q0 + q < n1) {
                            if constexpr (OP == kBgFp16) {
                                d1[0] = mfma_op<OP>(w1[q][0], e1[q], d1[0]);
                                d1[0] = mfma_op<OP>(w1[q][1], e1[q], d1[0]);
                            } else {
#pragma unroll
                                for (int h = 0; h < NTERM; ++h) d1[h] = mfma_op<OP>(w1[q][h], e1[q], d1[h]);
                            }
                        }
                    }
                }
                // D lane l: cells 4 (l / 16) + e of the tile, column l % 16
                const int ucol = l16 / (2 * P);
                if (ucol < nb) {
                    const int p = (P == 2) ? ((l16 >> 1) & 1) : 0;
                    const int ri = l16 & 1;
                    _Float16* dst = s_A1 + (ucol * M1 + p * R4) * A1P + ri * KPAD;
                    auto store = [&](int i, const floatx4 (&d)[NTERM]) {
                        const uint2 cw =
                            *reinterpret_cast<const uint2*>(a.cells + ((size_t)bc.tile_off + i) * 16 + 4 * l4);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint32_t cv = ((e < 2) ? cw.x : cw.y) >> (16 * (e & 1)) & 0xFFFFu;
                            float val = d[0][e];
                            if constexpr (OP == kBgFp8)
                                val = fmaf(fmaf(d[2][e], 0.0625f, d[1][e]), 0.0625f, d[0][e]) * inv_scale;
                            if (cv != 0xFFFFu) dst[(int)(cv >> 8) * A1P + (int)(cv & 0xFFu)] = (_Float16)val;
                        }
                    };
                    store(i0, d0);
                    if (i1 < bc.n_tile) store(i1, d1);
                }
            }
            __syncthreads();
            // 1'. decode the next step's spectra (the field operand is free now)
            if (u0 + a.TB < n) decode(c, t + u0 + a.TB, (int)std::min<int64_t>(a.TB, n - u0 - a.TB));
            // row-pass operand of this wave (L2-resident; loaded per step so that
            // its registers are free during the gridding product)
            half8 b1[Sh::NT1][Sh::KK];
            load_row_fragments<Sh>(b1, a.dft, kpart, mw, l16, l4);
            for (int u = 0; u < nb; ++u) {
                __builtin_amdgcn_s_setprio(1);
                row_pass<Sh, P>(s_A1 + u * M1 * A1P, s_B2, b1, M1, R4, mw, l16, l4);
                __syncthreads();
                __builtin_amdgcn_s_setprio(0);
                col_pass<Sh, P>(s_B2, a2, acc, l16, l4);
                // the next row pass overwrites B2; the next gridding product
                // touches neither B2 nor anything the column pass reads
                if (u + 1 < nb) __syncthreads();
            }
        }
        flush_slot<Sh, P>(a.slots, slot, a.C, c, kpart, acc, mw, l16, l4, a.fresh != 0);
        f += n;
        ++s_ch;
        v += KS;
        t = 0;
    }
}

// FP8 weight scale: the largest |w| of the sub-array's entries (a grid-stride
// maximum per workgroup, combined with an integer maximum on the float bits,
// which order like the values for |w| >= 0), then scale = 2^e with
// 224 <= s max|w| < 448 and its inverse.
__global__ void bg_absmax_kernel(const float* __restrict__ grp_w, int64_t n, unsigned int* __restrict__ bits) {
    __shared__ float red[256];
    float m = 0.f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(grp_w[k]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(bits, __float_as_uint(red[0]));
}

__global__ void bg_scale_kernel(float* __restrict__ scale) {
    if (threadIdx.x != 0) return;
    const float mx0 = __uint_as_float(reinterpret_cast<unsigned int*>(scale)[0]);
    const float mx = mx0 > 0.f ? mx0 : 1.f;
    const int e = (int)floorf(log2f(224.f / mx));
    scale[0] = ldexpf(1.f, e);
    scale[1] = ldexpf(1.f, -e);
}

// Split every gather entry's weight w into the operand parts of its block
// element (term t at w8 + t * term_elems): FP16 hi = fp16(w), lo = fp16(w - hi);
// FP8 r0 = s w, part t = e4m3(r_t), r_{t+1} = 16 (r_t - part t), t = 0, 1, 2.
// Padding entries (dst < 0) are skipped; elements no entry maps to stay zero.
template <int OP>
__global__ void bg_weights_kernel(const float* __restrict__ grp_w, const int32_t* __restrict__ dst, int64_t n,
                                  const float* __restrict__ scale, unsigned char* __restrict__ w8,
                                  int64_t term_elems) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t d = dst[k];
    if (d < 0) return;
    const float w = grp_w[k];
    if constexpr (OP == kBgFp16) {
        _Float16* wh = reinterpret_cast<_Float16*>(w8);
        const _Float16 h = (_Float16)w;
        wh[d] = h;
        wh[term_elems + d] = (_Float16)(w - (float)h);
    } else {
        float r = w * scale[0];
        for (int t = 0; t < 3; ++t) {
            const int b = __builtin_amdgcn_cvt_pk_fp8_f32(r, 0.0f, 0, false);
            w8[t * term_elems + d] = (unsigned char)(b & 0xFF);
            r = (r - __builtin_amdgcn_cvt_f32_fp8(b, 0)) * 16.0f;
        }
    }
}

// ---- launch shapes -----------------------------------------------------------
struct BgLayout {
    uint32_t off_E, off_A1, off_B2;
    int A1rows;
    size_t total;
};

size_t take16(size_t& b, size_t n) {
    b = (b + 15) & ~(size_t)15;
    const size_t o = b;
    b += n;
    return o;
}

BgLayout bg_layout(const SubDev& d, int TB) {
    BgLayout L{};
    size_t b = 0;
    const int eb = d.precision == EPIC_FP8 ? 1 : 2;
    const int K2 = 32 * d.KK;
    const int NK = d.N / (d.N > 64 ? 2 : 1);
    L.A1rows = TB * d.P * d.R4max + 16;
    L.off_E = (uint32_t)take16(b, (size_t)d.bg_nablk * 64 * 8 * eb);
    L.off_A1 = (uint32_t)take16(b, (size_t)L.A1rows * (K2 + kPadH) * 2);
    L.off_B2 = (uint32_t)take16(b, (size_t)d.P * NK * (K2 + kPadH) * 2);
    L.total = (b + 15) & ~(size_t)15;
    return L;
}

using BgFn = void (*)(BgArgs);

template <int N, int KK>
BgFn bg_pick2(int P, int op) {
    if (P == 2) return op == kBgFp8 ? bg_kernel<N, KK, 2, kBgFp8> : bg_kernel<N, KK, 2, kBgFp16>;
    return op == kBgFp8 ? bg_kernel<N, KK, 1, kBgFp8> : bg_kernel<N, KK, 1, kBgFp16>;
}

BgFn bg_select(int N, int KK, int P, int op) {
    switch (N * 8 + KK) {
#define EPIC_BG(NN, KKK) case NN * 8 + KKK: return bg_pick2<NN, KKK>(P, op);
        EPIC_BG(32, 1) EPIC_BG(32, 2)
        EPIC_BG(48, 1) EPIC_BG(48, 2) EPIC_BG(48, 3)
        EPIC_BG(64, 1) EPIC_BG(64, 2) EPIC_BG(64, 3) EPIC_BG(64, 4)
        EPIC_BG(96, 1) EPIC_BG(96, 2) EPIC_BG(96, 3) EPIC_BG(96, 4)
        EPIC_BG(128, 1) EPIC_BG(128, 2) EPIC_BG(128, 3) EPIC_BG(128, 4)
#undef EPIC_BG
    }
    return nullptr;
}

constexpr size_t kLdsLimit = 160 * 1024;

int op_of(const SubDev& d) { return d.precision == EPIC_FP8 ? kBgFp8 : kBgFp16; }

}  // namespace

// Launch shape of the GEMM-gridding form: the same grids and column split as
// the gather form; TB spectra per gridding step, the most of 16 / (2 P),
// 8 / (2 P), ... whose LDS lets the shape's target workgroups share a CU
// (two for N <= 64 with at most two MFMA steps, as the registers allow, else
// one).
hipError_t bg_configure(SubDev& d, int device, int num_cu, int force_tb) {
    const int need = std::max(d.Rmax, d.Wmax);
    d.KK = (need + 15) / 16;
    if (d.N < 32 || d.N > 128 || d.N % 16 != 0 || d.N == 80 || d.N == 112) return hipErrorNotSupported;
    if (d.KK < 1 || 16 * d.KK > d.N || d.KK > 4) return hipErrorNotSupported;
    if (!(d.wmode == kWShared || (d.P == 1 && d.wmode == kWReal))) return hipErrorNotSupported;
    d.KS = d.N > 64 ? 2 : 1;
    d.threads = 64 * (d.N / 16);
    const int target = (d.N <= 64 && d.KK <= 2) ? 2 : 1;   // workgroups per CU the registers allow
    const int tbmax = 16 / (2 * d.P);
    int tb = 0;
    for (int cand = tbmax; cand >= 1 && tb == 0; cand /= 2)
        if (bg_layout(d, cand).total <= kLdsLimit / target) tb = cand;
    for (int cand = tbmax; cand >= 1 && tb == 0; cand /= 2)
        if (bg_layout(d, cand).total <= kLdsLimit) tb = cand;
    if (tb == 0) return hipErrorNotSupported;
    if (force_tb > 0) {   // a candidate of the autotuner: any step size whose LDS fits
        if (force_tb > tbmax || bg_layout(d, force_tb).total > kLdsLimit) return hipErrorNotSupported;
        tb = force_tb;
    }
    d.bg_tb = tb;
    const BgLayout L = bg_layout(d, tb);
    d.lds_bytes = L.total;
    d.prog_lds = 0;
    int occ = 1;
    if (device >= 0) {
        BgFn fn = bg_select(d.N, d.KK, d.P, op_of(d));
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

hipError_t launch_bg_weights(const SubDev& d, hipStream_t st) {
    const int64_t n = d.bg_nentries;   // gather entries
    if (d.precision == EPIC_FP8) {
        unsigned int* bits = reinterpret_cast<unsigned int*>(d.bg_scale);
        hipError_t e = launch_zero(d.bg_scale, 1, st);   // the maximum's bits start at +0
        if (e != hipSuccess) return e;
        const int64_t nb = std::min<int64_t>(1024, (n + 255) / 256);
        bg_absmax_kernel<<<dim3((unsigned)std::max<int64_t>(1, nb)), dim3(256), 0, st>>>(d.grp_w, n, bits);
        bg_scale_kernel<<<dim3(1), dim3(64), 0, st>>>(d.bg_scale);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int bs = 256;
    const dim3 grid((unsigned)((n + bs - 1) / bs));
    const int64_t term_elems = d.bg_nent * 512;
    if (d.precision == EPIC_FP8)
        bg_weights_kernel<kBgFp8><<<grid, dim3(bs), 0, st>>>(d.grp_w, d.bg_dst, n, d.bg_scale, d.bg_w, term_elems);
    else
        bg_weights_kernel<kBgFp16><<<grid, dim3(bs), 0, st>>>(d.grp_w, d.bg_dst, n, d.bg_scale, d.bg_w, term_elems);
    return hipGetLastError();
}

hipError_t launch_bgemm(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st) {
    const BgLayout L = bg_layout(d, d.bg_tb);
    BgArgs a{};
    a.samples = samples;
    a.chans = d.chans;
    a.bg = d.bg_chans;
    a.tiles = d.bg_tiles;
    a.cells = d.bg_cells;
    a.ents = d.bg_ents;
    a.perm = d.bg_perm;
    a.w = d.bg_w;
    a.wterm = d.bg_nent * 512 * (d.precision == EPIC_FP8 ? 1 : 2);
    a.scale = d.bg_scale;
    a.dft = reinterpret_cast<const _Float16*>(d.dft16);
    a.slots = d.slots;
    a.fresh = d.fresh;
    a.T = n_time;
    a.C = d.C; a.A = d.A; a.nibble_order = d.nibble_order; a.TB = d.bg_tb; a.nablk = d.bg_nablk;
    a.V = d.C * d.KS;
    a.off_E = L.off_E; a.off_A1 = L.off_A1; a.off_B2 = L.off_B2;
    a.A1rows = L.A1rows;
    a.grid_wg = d.grid_wg;
    a.wg_per_xcd = (d.grid_wg + 7) / 8;
    BgFn fn = bg_select(d.N, d.KK, d.P, op_of(d));
    if (!fn) return hipErrorNotSupported;
    hipLaunchKernelGGL(fn, dim3(8 * a.wg_per_xcd), dim3(d.threads), L.total, st, a);
    return hipGetLastError();
}

}  // namespace epic
