// FP32 hot path: one persistent fused kernel per sub-array.  Each workgroup
// takes an equal, contiguous run of the (channel, spectrum) sequence and, for
// each spectrum,
//   1. decodes the A*P 4+4-bit samples into LDS                 (Sec. 2.1)
//   2. grids them by gathering, per non-empty aperture cell, the weighted
//      samples of every antenna whose kernel covers the cell     (Eq. 4, Sec. 3.1)
//   3. transforms the aperture window along x (rows), then along y (columns),
//      with exp(+2 pi i ...) N-point DFTs                        (Eq. 4)
//   4. forms XX*, YY*, Re XY*, Im XY* per pixel and adds them into registers
//                                                               (Eq. 5, Sec. 3.2)
// and when its run leaves a channel (or ends) adds the registers into that
// channel's partial-accumulator slot.  Slots are summed in a fixed order by
// the read-out, so results are bitwise reproducible.
//
// Transform layout.  N = 8 Q.  Every N-point DFT is split as
//   X[q + Q m] = sum_{n1<8} w_N^{n1 q} [ sum_{n2} v[n1 + 8 n2] w_Q^{n2 q} ] w_8^{n1 m},
// so lane (q, k) folds its input column with per-lane twiddles and finishes
// with a register 8-point DFT, producing the 8 outputs j = q + Q m.  Only the
// R x W aperture window is non-zero, so the row pass runs on R rows only and
// both passes fold just R (or W) inputs.  The column pass leaves each pixel's
// X and Y values in the same lane, so the products and the time accumulation
// never leave registers: 8 pixels x 4 products per lane.
//
// Large grids split the image columns over KS workgroups by q: part k takes
// q in [k Q/KS, (k+1) Q/KS), i.e. the columns j = q + Q m of those q, so each
// part row-transforms only its own q values (the row pass is not repeated per
// part; the decode and the gridding are).
//
// The window sits at the grid origin instead of at its absolute cells, and the
// (-1)^(x+y) image-centring factor is replaced by reading bin (i + N/2) mod N
// for pixel i: both only multiply X and Y by one common unit phase, which the
// products of Eq. 5 cancel.
#include <hip/hip_runtime.h>

#include "epic_device.hpp"
#include "epic_gather.hpp"
#include "epic_internal.hpp"
#include "epic_sched.hpp"

namespace epic {

namespace {

struct Fp32Args {
    const uint8_t* samples;   // [T][C][A][P]
    int64_t T;
    int C, A, S;
    const ChanInfo* chans;
    const CellDesc* cells_desc;
    const uint2* grp_ant;     // 4 x u16 per group
    const float4* grp_w;      // weights per group (1, 2 or 4 float4)
    const float2* twiddle;    // [N]
    float* slots;             // [S][C][NPP][N][N]
    float2* efield;           // E-field form: [T][C][P][N][N] output images
    int Rmax, WP;             // window rows (padded), gather-program row pitch
    uint32_t off_w, off_gant, off_desc, off_smp, off_G, off_Y, off_tw, off_tq;
    int nibble_order;
    int dbuf;                 // 1: two sample buffers (decode overlaps gridding)
    int fresh;                // 1: the slots hold zeros, store instead of add
    int grid_wg, wg_per_xcd;
};

template <int N_>
struct Shape {
    static constexpr int N = N_;
    static constexpr int Q = N / 8;                            // lanes per image column
    // image columns split over KS workgroups (1, 2, 4 or 8) so that a
    // workgroup holds at most 1024 (q, column) lanes
    static constexpr int KS = (Q * N <= 1024) ? 1 : (Q * N <= 2048 ? 2 : (Q * N <= 4096 ? 4 : 8));
    static constexpr int NK = N / KS;                          // columns per workgroup
    static constexpr int QS = Q / KS;                          // row-pass q values per workgroup
    static_assert(Q % KS == 0, "the column parts split q evenly");
    static constexpr int LANES = Q * NK;                       // (q, column) lanes
    static constexpr int THREADS = ((LANES + 63) / 64) * 64;
    // register budget: two 8-wave workgroups per CU (<= 128 VGPRs); larger
    // workgroups just have to fit once; smaller ones are left to the compiler
    static constexpr int WAVES = THREADS / 64;
    static constexpr int MIN_WAVES_PER_EU = WAVES == 8 ? 4 : (WAVES > 8 ? (WAVES + 3) / 4 : 1);
};

constexpr int kPrefetch = 1;   // sample words per thread held in registers ahead of use (more are loaded directly)

// ---- DFT input fold ---------------------------------------------------------
// z[n1] = w_N^{n1 q} * sum_{n2 < nb} v[(n1 + 8 n2) * STRIDE] * w_Q^{n2 q} over
// the len non-zero inputs, nb = ceil(len / 8).  The window is zero-padded to
// whole blocks of 8, so the first block is a plain load and no block needs a
// bounds check; of the last block only its first 1, 2, 4 or 8 inputs (the
// non-zero part, rounded up) are folded.  Control flow depends only on len
// (uniform).
// tq is the lane's row of the LDS table of per-q factors: tq[n1] = w_N^{n1 q}
// (n1 < 8) and tq[8 + n2] = w_Q^{n2 q} (n2 < Q), so every factor is a load at a
// constant offset from one address.  tw holds w_N^{n1 q} in registers; with
// TW_LDS the twiddles are read from tq instead and tw is unused.
//
// Windows of two or three blocks (the common case) take fold_fixed, which
// issues every LDS load of the fold before its first product, so a lane
// waits for LDS once per fold rather than once per block.
template <int N, bool TW_LDS, int STRIDE, int NB, int LAST>
__device__ __forceinline__ void fold_fixed(float2 (&z)[8], const float2* __restrict__ v, const float2 (&tw)[8],
                                           const float2* __restrict__ tq) {
    float2 b[NB - 1][8], w[NB - 1], t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) z[k] = v[k * STRIDE];
#pragma unroll
    for (int n2 = 1; n2 < NB; ++n2) {
        w[n2 - 1] = tq[8 + n2];
#pragma unroll
        for (int k = 0; k < ((n2 == NB - 1) ? LAST : 8); ++k) b[n2 - 1][k] = v[(8 * n2 + k) * STRIDE];
    }
    if constexpr (TW_LDS) {
#pragma unroll
        for (int n1 = 1; n1 < 8; ++n1) t[n1] = tq[n1];
    }
#pragma unroll
    for (int n2 = 1; n2 < NB; ++n2)
#pragma unroll
        for (int k = 0; k < ((n2 == NB - 1) ? LAST : 8); ++k) z[k] = cfma(z[k], b[n2 - 1][k], w[n2 - 1]);
#pragma unroll
    for (int n1 = 1; n1 < 8; ++n1) z[n1] = cmul(z[n1], TW_LDS ? t[n1] : tw[n1]);   // w^0 = 1
}

template <int N, bool TW_LDS, int STRIDE, bool FIXED>
__device__ __forceinline__ void fold_twiddle(float2 (&z)[8], const float2* __restrict__ v, int len,
                                             const float2 (&tw)[8], const float2* __restrict__ tq) {
    const int nb = (len + 7) >> 3;
    const int tail = len - 8 * (nb - 1);   // non-zero inputs of the last block, 1..8
    if (FIXED && nb == 3) {
        if (tail <= 1) fold_fixed<N, TW_LDS, STRIDE, 3, 1>(z, v, tw, tq);
        else if (tail <= 2) fold_fixed<N, TW_LDS, STRIDE, 3, 2>(z, v, tw, tq);
        else if (tail <= 4) fold_fixed<N, TW_LDS, STRIDE, 3, 4>(z, v, tw, tq);
        else fold_fixed<N, TW_LDS, STRIDE, 3, 8>(z, v, tw, tq);
        return;
    }
    if (FIXED && nb == 2) {
        if (tail <= 1) fold_fixed<N, TW_LDS, STRIDE, 2, 1>(z, v, tw, tq);
        else if (tail <= 2) fold_fixed<N, TW_LDS, STRIDE, 2, 2>(z, v, tw, tq);
        else if (tail <= 4) fold_fixed<N, TW_LDS, STRIDE, 2, 4>(z, v, tw, tq);
        else fold_fixed<N, TW_LDS, STRIDE, 2, 8>(z, v, tw, tq);
        return;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) z[k] = v[k * STRIDE];
    // not unrolled: an unrolled loop lets the compiler hoist every block's LDS
    // loads above the exit test, which costs ~100 registers
#pragma unroll 1
    for (int n2 = 1; n2 < nb - 1; ++n2) {
        const float2 w = tq[8 + n2];
        const float2* vb = v + 8 * n2 * STRIDE;
#pragma unroll
        for (int k = 0; k < 8; ++k) z[k] = cfma(z[k], vb[k * STRIDE], w);
    }
    if (nb >= 2) {
        const float2 w = tq[8 + nb - 1];
        const float2* vb = v + 8 * (nb - 1) * STRIDE;
        z[0] = cfma(z[0], vb[0], w);
        if (tail > 1) z[1] = cfma(z[1], vb[STRIDE], w);
        if (tail > 2) {
            z[2] = cfma(z[2], vb[2 * STRIDE], w);
            z[3] = cfma(z[3], vb[3 * STRIDE], w);
        }
        if (tail > 4) {
#pragma unroll
            for (int k = 4; k < 8; ++k) z[k] = cfma(z[k], vb[k * STRIDE], w);
        }
    }
#pragma unroll
    for (int n1 = 1; n1 < 8; ++n1) z[n1] = cmul(z[n1], TW_LDS ? tq[n1] : tw[n1]);   // w^0 = 1
}

// EF: write each spectrum's transformed fields (X, Y) to a.efield instead of
// accumulating their products.
template <int N_, int P, int WM, bool PROG_LDS, bool EF = false>
__global__ void __launch_bounds__(Shape<N_>::THREADS)
    __attribute__((amdgpu_waves_per_eu(Shape<N_>::MIN_WAVES_PER_EU))) fp32_kernel(Fp32Args a) {
    using Sh = Shape<N_>;
    constexpr int N = Sh::N, Q = Sh::Q, KS = Sh::KS, NK = Sh::NK, LANES = Sh::LANES, THREADS = Sh::THREADS;
    constexpr int NPP = (P == 2) ? 4 : 1;
    constexpr int GF4 = group_f4<P, WM>();
    const int tid = threadIdx.x;

    // Persistent, XCD-aware: consecutive runs (mostly the same channel) share
    // an XCD and its L2.
    const int b = blockIdx.x;
    const int g = (b & 7) * a.wg_per_xcd + (b >> 3);
    if (g >= a.grid_wg) return;
    const int64_t T = a.T;
    const PartSplit ps = part_split(g, a.grid_wg, KS);
    const int kpart = ps.kpart;
    const int64_t total = (int64_t)a.C * T;   // this column part's (channel, spectrum) sequence
    const int64_t L = (total + ps.Gp - 1) / ps.Gp;
    int64_t f0, f1;
    owned_range(ps.gp, L, 0, 1, total, &f0, &f1);
    if (f0 >= f1) return;

    extern __shared__ __align__(16) unsigned char smem[];
    float4* s_w = reinterpret_cast<float4*>(smem + a.off_w);
    uint2* s_gant = reinterpret_cast<uint2*>(smem + a.off_gant);
    uint2* s_desc = reinterpret_cast<uint2*>(smem + a.off_desc);
    // one or two sample buffers, FP16 (exact for 4-bit values; the gather's
    // FMAs convert on the fly, and the LDS reads are half as wide)
    h2v* s_smp0 = reinterpret_cast<h2v*>(smem + a.off_smp);
    h2v* s_smp1 = a.dbuf ? s_smp0 + a.A * P : s_smp0;
    float2* s_G = reinterpret_cast<float2*>(smem + a.off_G);
    float2* s_Y = reinterpret_cast<float2*>(smem + a.off_Y);
    float2* s_tw = reinterpret_cast<float2*>(smem + a.off_tw);
    for (int k = tid; k < N; k += THREADS) s_tw[k] = a.twiddle[k];
    // per-q factor rows: [w_N^{n1 q}, n1 < 8 | w_Q^{n2 q} = w_N^{8 n2 q}, n2 < Q]
    constexpr int TQP = 8 + N / 8;
    float2* s_tq = reinterpret_cast<float2*>(smem + a.off_tq);
    for (int k = tid; k < (N / 8) * TQP; k += THREADS) {
        const int qq = k / TQP, j = k - qq * TQP;
        s_tq[k] = a.twiddle[(j < 8 ? j * qq : 8 * (j - 8) * qq) % N];
    }

    // per-lane transform constants (q is wave-uniform when a wave holds one q)
    const bool lane_on = tid < LANES;
    int q = lane_on ? tid / NK : 0;
    if constexpr (NK % 64 == 0) q = __builtin_amdgcn_readfirstlane(q);
    const int kk = lane_on ? tid - q * NK : 0;
    float2 tw[8];
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) tw[n1] = a.twiddle[(n1 * q) % N];
    constexpr int QS = Sh::QS;
    constexpr int YP = NK + 1;   // s_Y row pitch (float2), as laid out on the host
    // grids up to 64: windows of at most a few blocks, folded with every load
    // issued up front (rows), and the column lanes' twiddles read from LDS
    // (q is wave-uniform there) to leave the registers to those loads
    constexpr bool kSmallGrid = N <= 64;
    // image column of local column kk
    auto column_of = [&](int k) {
        if constexpr (KS == 1) return k;
        return kpart * QS + k % QS + Q * (k / QS);
    };

    const int AP = a.A * P;
    const bool words = ((AP & 3) == 0) && ((reinterpret_cast<uintptr_t>(a.samples) & 3) == 0);
    // decoding runs on the workgroup's last lanes: the gather cells are sorted
    // by group count, so the first waves carry the longest gather chains
    const int dtid = THREADS - 1 - tid;
    const int nwords = AP >> 2;

    uint32_t pre[kPrefetch];   // the next spectrum's sample words, loaded ahead of use
    auto prefetch = [&](int vv, int64_t tt) {   // vv: channel
        const uint32_t* row4 =
            reinterpret_cast<const uint32_t*>(a.samples + ((int64_t)tt * a.C + vv) * AP);
#pragma unroll
        for (int k = 0; k < kPrefetch; ++k) {
            const int w = dtid + k * THREADS;
            pre[k] = (w < nwords) ? row4[w] : 0u;
        }
    };

    // decode one (t, c) row of A*P bytes into dst: the prefetched words first,
    // any further words straight from memory
    auto decode = [&](h2v* dst, int cc, int64_t tt) {
        if (words) {
#pragma unroll
            for (int k = 0; k < kPrefetch; ++k) {
                const int w = dtid + k * THREADS;
                if (w < nwords) {
                    const uint32_t x = pre[k];
                    dst[4 * w + 0] = unpack44_h(x & 0xFFu, a.nibble_order);
                    dst[4 * w + 1] = unpack44_h((x >> 8) & 0xFFu, a.nibble_order);
                    dst[4 * w + 2] = unpack44_h((x >> 16) & 0xFFu, a.nibble_order);
                    dst[4 * w + 3] = unpack44_h(x >> 24, a.nibble_order);
                }
            }
            const uint32_t* row4 = reinterpret_cast<const uint32_t*>(a.samples + ((int64_t)tt * a.C + cc) * AP);
            for (int w = dtid + kPrefetch * THREADS; w < nwords; w += THREADS) {
                const uint32_t x = row4[w];
                dst[4 * w + 0] = unpack44_h(x & 0xFFu, a.nibble_order);
                dst[4 * w + 1] = unpack44_h((x >> 8) & 0xFFu, a.nibble_order);
                dst[4 * w + 2] = unpack44_h((x >> 16) & 0xFFu, a.nibble_order);
                dst[4 * w + 3] = unpack44_h(x >> 24, a.nibble_order);
            }
        } else {
            const uint8_t* row = a.samples + ((int64_t)tt * a.C + cc) * AP;
            for (int k = dtid; k < AP; k += THREADS) dst[k] = unpack44_h(row[k], a.nibble_order);
        }
    };

    int v = (int)(f0 / T);   // channel
    int64_t t = f0 - (int64_t)v * T;
    if (words) prefetch(v, t);
    for (int64_t f = f0; f < f1;) {
        // one channel segment: spectra t .. t+n-1 of channel v
        const int64_t n = (f1 - f < T - t) ? f1 - f : T - t;
        const int c = v;
        const int slot = slot_of(ps.gp, v, t, T, 0, 1, L);
        const ChanInfo ci = a.chans[c];
        const int R = ci.R, W = ci.W, n_cell = ci.n_cell;
        const int PR = P * R;
        const float inv_pr = 1.0f / (float)PR;
        // the lane's first row-pass task (tau = tid) for the whole segment
        int qi_0 = (int)((float)tid * inv_pr);
        int rr_0 = tid - qi_0 * PR;
        if (rr_0 >= PR) {
            ++qi_0;
            rr_0 -= PR;
        }
        const CellDesc* g_desc = a.cells_desc + ci.cell_off;
        const uint2* g_gant = a.grp_ant + ci.grp_off;
        const float4* g_w = a.grp_w + (int64_t)ci.grp_off * GF4;
        __syncthreads();   // the previous segment is done with every LDS buffer
        if constexpr (PROG_LDS) {
            for (int k = tid; k < ci.n_grp * GF4; k += THREADS) s_w[k] = g_w[k];
            for (int k = tid; k < ci.n_grp; k += THREADS) s_gant[k] = g_gant[k];
            for (int k = tid; k < n_cell; k += THREADS) s_desc[k] = g_desc[k];
        }
        // zero the window buffers: cells beyond W (and rows beyond R) up to
        // the next multiple of 8 are read by the folds and must be zero
        for (int k = tid; k < P * a.Rmax * a.WP; k += THREADS) s_G[k] = make_float2(0.f, 0.f);
        for (int k = tid; k < P * a.Rmax * YP; k += THREADS) s_Y[k] = make_float2(0.f, 0.f);
        float acc[8][NPP];
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int k = 0; k < NPP; ++k) acc[m][k] = 0.f;

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
            h2v* s_smp = (i & 1) ? s_smp1 : s_smp0;
            h2v* s_nxt = (i & 1) ? s_smp0 : s_smp1;

            // Wave priorities: the gathering and the row pass are chains of
            // dependent LDS reads run by few waves, the column pass is VALU
            // work on every wave; raising the first two lets a CU's other
            // workgroup fill their gaps without delaying them.
            __builtin_amdgcn_s_setprio(2);
            // 2. gather gridding of the non-empty cells, both pols per cell
            for (int k = tid; k < n_cell; k += THREADS) {
                const uint2 d = PROG_LDS ? s_desc[k] : g_desc[k];
                const int off = (int)(d.x & 0xFFFFu);
                const int ng = (int)(d.x >> 16);
                float2 gx = make_float2(0.f, 0.f), gy = make_float2(0.f, 0.f);
                for (int j = 0; j < ng; ++j) {
                    const int gg = (int)d.y + j;
                    const uint2 ia = PROG_LDS ? s_gant[gg] : g_gant[gg];
                    const float4* w = PROG_LDS ? s_w + gg * GF4 : g_w + (int64_t)gg * GF4;
                    gather_group<P, WM>(gx, gy, w, ia, s_smp);
                }
                s_G[off] = gx;
                if constexpr (P == 2) s_G[a.Rmax * a.WP + off] = gy;
            }
            // 1'. decode the next spectrum of this segment into the other buffer
            if (a.dbuf && i + 1 < n) {
                decode(s_nxt, c, tt + 1);
                if (words && f + i + 2 < f1) {
                    if (tt + 2 < T) prefetch(v, tt + 2);
                    else prefetch(v + 1, 0);
                }
            }
            __syncthreads();

            __builtin_amdgcn_s_setprio(1);
            // 3a. row pass: the P R window rows x this part's QS values of q,
            //     packed densely onto the lanes (task tau = qi P R + row);
            //     local column qi + QS m holds image column qr + Q m
            for (int tau = tid; tau < PR * QS; tau += THREADS) {
                // tau / PR through the segment's reciprocal: tau < 2^14 and
                // PR <= 512, so the product is never high and at most one low
                int qi = qi_0, rr = rr_0;
                if (tau != tid) {
                    qi = (int)((float)tau * inv_pr);
                    rr = tau - qi * PR;
                    if (rr >= PR) {
                        ++qi;
                        rr -= PR;
                    }
                }
                const int qr = kpart * QS + qi;
                const int p = (P == 2 && rr >= R) ? 1 : 0;
                const int r = rr - p * R;
                float2 z[8];
                fold_twiddle<N, true, 1, kSmallGrid>(z, s_G + (p * a.Rmax + r) * a.WP, W, tw, s_tq + qr * TQP);
                fft8(z);
                float2* yrow = s_Y + (p * a.Rmax + r) * YP + qi;
#pragma unroll
                for (int m = 0; m < 8; ++m) yrow[QS * m] = z[fft8_pos(m)];
            }
            __syncthreads();

            // 1'. with one sample buffer the next spectrum is decoded here, after
            //     every gather read of the current one
            if (!a.dbuf && i + 1 < n) {
                decode(s_nxt, c, tt + 1);
                if (words && f + i + 2 < f1) {
                    if (tt + 2 < T) prefetch(v, tt + 2);
                    else prefetch(v + 1, 0);
                }
            }

            // 3b'. E-field form: each pixel's field, with the phase that moves the
            //      window from the grid origin back to its cells, e^{+2 pi i (x0 kx + y0 ky)/N}
            //      (the (-1)^(x+y) centring is the read of bin (i + N/2) mod N)
            if constexpr (EF) {
                if (lane_on) {
                    const int kx = column_of(kk);
                    int ii = kx + N / 2;
                    if (ii >= N) ii -= N;
                    const int rx = (ci.x0 * kx) % N;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        float2 X[8];
                        fold_twiddle<N, kSmallGrid, YP, false>(X, s_Y + p * a.Rmax * YP + kk, R, tw, s_tq + q * TQP);
                        fft8(X);
                        float2* out = a.efield + ((tt * a.C + c) * P + p) * (int64_t)N * N;
#pragma unroll
                        for (int m = 0; m < 8; ++m) {
                            const int ky = q + Q * m;
                            int jj = ky + N / 2;
                            if (jj >= N) jj -= N;
                            const float2 ph = s_tw[(rx + ci.y0 * ky) % N];
                            out[jj * N + ii] = cmul(X[fft8_pos(m)], ph);
                        }
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
            // 3b + 4. column pass per pol, products and accumulation in registers
            if (!EF && lane_on) {
                float2 X[8];
                fold_twiddle<N, kSmallGrid, YP, false>(X, s_Y + kk, R, tw, s_tq + q * TQP);
                fft8(X);
                if constexpr (P == 2) {
                    float2 Yv[8];
                    fold_twiddle<N, kSmallGrid, YP, false>(Yv, s_Y + a.Rmax * YP + kk, R, tw, s_tq + q * TQP);
                    fft8(Yv);
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        const float2 x = X[fft8_pos(m)], y = Yv[fft8_pos(m)];
                        acc[m][0] = fmaf(x.x, x.x, fmaf(x.y, x.y, acc[m][0]));
                        acc[m][1] = fmaf(y.x, y.x, fmaf(y.y, y.y, acc[m][1]));
                        acc[m][2] = fmaf(x.x, y.x, fmaf(x.y, y.y, acc[m][2]));
                        acc[m][3] = fmaf(x.y, y.x, fmaf(-x.x, y.y, acc[m][3]));
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        const float2 x = X[fft8_pos(m)];
                        acc[m][0] = fmaf(x.x, x.x, fmaf(x.y, x.y, acc[m][0]));
                    }
                }
            }
            // the next spectrum's decode barrier orders these LDS reads before
            // the next row pass overwrites s_Y; with one sample buffer this one
            // orders the decode above before the next gather
            if (!a.dbuf) __syncthreads();
        }

        // add the segment's sums into its slot; bin (k', j') -> pixel (+N/2 mod N)
        if (!EF && lane_on) {
            const int kb = column_of(kk);
            int ii = kb + N / 2;
            if (ii >= N) ii -= N;
            float* base = a.slots + ((int64_t)slot * a.C + c) * NPP * N * N;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                int j = q + Q * m + N / 2;
                if (j >= N) j -= N;
#pragma unroll
                for (int k = 0; k < NPP; ++k) slot_put(&base[((int64_t)k * N + j) * N + ii], acc[m][k], a.fresh != 0);
            }
        }
        f += n;
        ++v;
        t = 0;
    }
}

struct Layout {
    uint32_t off_w, off_gant, off_desc, off_smp, off_G, off_Y, off_tw, off_tq;
    size_t total;
    int YP;
};

Layout layout(const SubDev& d, int KS, bool prog_lds, int bufs) {
    Layout L{};
    size_t b = 0;
    auto take = [&](size_t n) {
        b = (b + 15) & ~(size_t)15;
        size_t o = b;
        b += n;
        return (uint32_t)o;
    };
    const int gf4 = group_f4_of(d.P, d.wmode);
    L.YP = d.N / KS + 1;
    L.off_w = prog_lds ? take((size_t)d.Gmax * gf4 * 16) : 0;
    L.off_gant = prog_lds ? take((size_t)d.Gmax * 8) : 0;
    L.off_desc = prog_lds ? take((size_t)d.CellMax * 8) : 0;
    L.off_smp = take((size_t)bufs * d.A * d.P * 4);
    L.off_G = take((size_t)d.P * d.Rmax * d.WP * sizeof(float2));
    L.off_Y = take((size_t)d.P * d.Rmax * L.YP * sizeof(float2));
    L.off_tw = take((size_t)d.N * sizeof(float2));
    L.off_tq = take((size_t)(d.N / 8) * (8 + d.N / 8) * sizeof(float2));
    L.total = (b + 15) & ~(size_t)15;
    return L;
}

using KernelFn = void (*)(Fp32Args);

template <int N, int P, int WM, bool EF>
KernelFn pick_wm(bool prog) {
    return prog ? fp32_kernel<N, P, WM, true, EF> : fp32_kernel<N, P, WM, false, EF>;
}

template <int N, int P, bool EF>
KernelFn pick(int wm, bool prog) {
    if (wm == kWComplex) return pick_wm<N, P, kWComplex, EF>(prog);
    if constexpr (P == 2)
        if (wm == kWShared) return pick_wm<N, P, kWShared, EF>(prog);
    return pick_wm<N, P, kWReal, EF>(prog);
}

// Grid sizes with a kernel: multiples of 16 from 16 to 128, 192 and 256.
KernelFn select_kernel(int N, int P, int wm, bool prog, bool ef = false) {
    switch (N * 2 + (P - 1)) {
#define EPIC_CASE(NN)                                                                            \
    case NN * 2 + 0: return ef ? pick<NN, 1, true>(wm, prog) : pick<NN, 1, false>(wm, prog); \
    case NN * 2 + 1: return ef ? pick<NN, 2, true>(wm, prog) : pick<NN, 2, false>(wm, prog);
        EPIC_CASE(16) EPIC_CASE(32) EPIC_CASE(48) EPIC_CASE(64) EPIC_CASE(80) EPIC_CASE(96) EPIC_CASE(112)
        EPIC_CASE(128) EPIC_CASE(192) EPIC_CASE(256)
#undef EPIC_CASE
    }
    return nullptr;
}

int threads_for(int N) {
    switch (N) {
        case 16: return Shape<16>::THREADS;
        case 32: return Shape<32>::THREADS;
        case 48: return Shape<48>::THREADS;
        case 64: return Shape<64>::THREADS;
        case 80: return Shape<80>::THREADS;
        case 96: return Shape<96>::THREADS;
        case 112: return Shape<112>::THREADS;
        case 128: return Shape<128>::THREADS;
        case 192: return Shape<192>::THREADS;
        case 256: return Shape<256>::THREADS;
    }
    return 0;
}

int ks_for(int N) {
    switch (N) {
        case 16: return Shape<16>::KS;
        case 32: return Shape<32>::KS;
        case 48: return Shape<48>::KS;
        case 64: return Shape<64>::KS;
        case 80: return Shape<80>::KS;
        case 96: return Shape<96>::KS;
        case 112: return Shape<112>::KS;
        case 128: return Shape<128>::KS;
        case 192: return Shape<192>::KS;
        case 256: return Shape<256>::KS;
    }
    return 1;
}

constexpr size_t kLdsLimit = 160 * 1024;

}  // namespace

// Choose the launch shape.  The gather program lives in LDS when it fits next
// to the per-spectrum buffers, else it streams from L2.  The grid is one
// resident round of workgroups (occupancy x CUs).  device < 0: no HIP calls.
hipError_t fp32_configure(SubDev& d, int device, int num_cu) {
    if (threads_for(d.N) == 0) return hipErrorNotSupported;
    d.KS = ks_for(d.N);
    d.threads = threads_for(d.N);
    // two sample buffers unless only one fits
    d.smp_bufs = layout(d, d.KS, false, 2).total <= kLdsLimit ? 2 : 1;
    const Layout with = layout(d, d.KS, true, d.smp_bufs);
    const Layout without = layout(d, d.KS, false, d.smp_bufs);
    const bool prog = with.total <= kLdsLimit / 2 || (with.total <= kLdsLimit && without.total > kLdsLimit / 2);
    const Layout& L = prog ? with : without;
    if (L.total > kLdsLimit) return hipErrorNotSupported;
    d.lds_bytes = L.total;
    d.prog_lds = prog ? 1 : 0;
    int occ = 2;
    if (device >= 0) {
        KernelFn fn = select_kernel(d.N, d.P, d.wmode, prog);
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

hipError_t launch_fp32(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st, float* efield) {
    const bool prog = d.prog_lds != 0;
    const Layout L = layout(d, d.KS, prog, d.smp_bufs);
    Fp32Args a{};
    a.samples = samples;
    a.T = n_time;
    a.C = d.C; a.A = d.A; a.S = d.S;
    a.chans = d.chans;
    a.cells_desc = d.cells_desc;
    a.grp_ant = reinterpret_cast<const uint2*>(d.grp_ant);
    a.grp_w = reinterpret_cast<const float4*>(d.grp_w);
    a.twiddle = d.twiddle; a.slots = d.slots;
    a.efield = reinterpret_cast<float2*>(efield);
    a.Rmax = d.Rmax; a.WP = d.WP;
    a.off_w = L.off_w; a.off_gant = L.off_gant; a.off_desc = L.off_desc;
    a.off_smp = L.off_smp; a.off_G = L.off_G; a.off_Y = L.off_Y; a.off_tw = L.off_tw; a.off_tq = L.off_tq;
    a.nibble_order = d.nibble_order;
    a.dbuf = d.smp_bufs == 2 ? 1 : 0;
    a.fresh = d.fresh;
    a.grid_wg = d.grid_wg;
    a.wg_per_xcd = (d.grid_wg + 7) / 8;
    KernelFn fn = select_kernel(d.N, d.P, d.wmode, prog, efield != nullptr);
    if (!fn) return hipErrorNotSupported;
    if (efield) {   // the E-field instances get their LDS limit on first use
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(8 * a.wg_per_xcd), dim3(d.threads), L.total, st, a);
    return hipGetLastError();
}

}  // namespace epic
