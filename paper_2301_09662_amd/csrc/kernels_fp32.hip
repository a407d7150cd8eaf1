// FP32 hot path: one fused kernel per sub-array that, for each (channel, time
// slot) work item, loops over its spectra and for each spectrum
//   1. decodes the A*P 4+4-bit samples into LDS                 (Sec. 2.1)
//   2. grids them by gathering, per aperture cell, the weighted samples of
//      every antenna whose kernel covers the cell                (Eq. 4, Sec. 3.1)
//   3. transforms the aperture window along x (rows), then along y (columns),
//      with exp(+2 pi i ...) N-point DFTs                        (Eq. 4)
//   4. forms XX*, YY*, Re XY*, Im XY* per pixel and adds them into registers
//                                                               (Eq. 5, Sec. 3.2)
// and finally adds the registers into its slot of the partial accumulators.
//
// Transform layout.  N = 16 Q.  Every N-point DFT is split as
//   X[q + Q m] = sum_{n1<16} w_N^{n1 q} [ sum_{n2} v[n1 + 16 n2] w_Q^{n2 q} ] w_16^{n1 m},
// so lane (q, k) folds its input column with per-lane twiddles and finishes
// with a register 16-point DFT, producing the 16 outputs j = q + Q m.  Only the
// R x W aperture window is non-zero, so the row pass runs on R rows only and
// both passes fold just R (or W) inputs.  The column pass leaves each pixel's
// X and Y values in the same lane, so the products and the time accumulation
// never leave registers: 16 pixels x 4 products per lane.
//
// The window sits at the grid origin instead of at its absolute cells, and the
// (-1)^(x+y) image-centring factor is replaced by reading bin (i + N/2) mod N
// for pixel i: both only multiply X and Y by one common unit phase, which the
// products of Eq. 5 cancel.
#include <hip/hip_runtime.h>

#include "epic_device.hpp"
#include "epic_internal.hpp"

namespace epic {

namespace {

struct Fp32Args {
    const uint8_t* samples;   // [T][C][A][P]
    int64_t T;
    int C, A, S;
    const ChanInfo* chans;
    const uint32_t* cell_ptr;
    const uint16_t* ent_ant;
    const float* ent_w;
    const float2* twiddle;    // [N]
    float* slots;             // [S][C][NPP][N][N]
    int Rmax, WP, YP;
    uint32_t off_w, off_smp, off_G, off_Y, off_cp, off_ant;
    int nibble_order;
    int units, units_per_xcd;
};

template <int Q>
struct Shape {
    static constexpr int N = 16 * Q;
    static constexpr int KS = (Q >= 7) ? 2 : 1;        // image columns split over KS workgroups
    static constexpr int NK = N / KS;                  // columns per workgroup
    static constexpr int LANES = Q * NK;               // (q, column) lanes
    static constexpr int THREADS = ((LANES + 63) / 64) * 64;
};

// z[n1] = w_N^{n1 q} * sum_{n2} v[(n1 + 16 n2) * stride] * w_Q^{n2 q}, for the
// first `len` inputs (the rest are zero).  `len` is uniform across the block.
template <int Q>
__device__ __forceinline__ void fold_twiddle(float2 (&z)[16], const float2* __restrict__ v, int stride, int len,
                                             const float2 (&tw)[16], const float2 (&wq)[Q]) {
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
        float2 s = make_float2(0.f, 0.f);
        if (n1 < len) s = v[n1 * stride];
#pragma unroll
        for (int n2 = 1; n2 < Q; ++n2) {
            const int n = n1 + 16 * n2;
            if (n < len) s = cfma(s, v[n * stride], wq[n2]);
        }
        z[n1] = cmul(s, tw[n1]);
    }
}

template <int Q, int P, bool CSR_LDS>
__global__ void __launch_bounds__(Shape<Q>::THREADS) fp32_kernel(Fp32Args a) {
    using Sh = Shape<Q>;
    constexpr int N = Sh::N, KS = Sh::KS, NK = Sh::NK, LANES = Sh::LANES, THREADS = Sh::THREADS;
    constexpr int NPP = (P == 2) ? 4 : 1;
    const int tid = threadIdx.x;

    // XCD-aware work item: consecutive items (same channel) share an XCD's L2.
    const int b = blockIdx.x;
    const int u = (b & 7) * a.units_per_xcd + (b >> 3);
    if (u >= a.units) return;
    const int kpart = u % KS;
    const int cs = u / KS;
    const int s = cs % a.S;
    const int c = cs / a.S;
    const int64_t t0 = ((int64_t)s * a.T) / a.S;
    const int64_t t1 = ((int64_t)(s + 1) * a.T) / a.S;
    if (t0 >= t1) return;

    extern __shared__ __align__(16) unsigned char smem[];
    float* s_w = reinterpret_cast<float*>(smem + a.off_w);
    float2* s_smp = reinterpret_cast<float2*>(smem + a.off_smp);
    float2* s_G = reinterpret_cast<float2*>(smem + a.off_G);
    float2* s_Y = reinterpret_cast<float2*>(smem + a.off_Y);
    uint32_t* s_cp = reinterpret_cast<uint32_t*>(smem + a.off_cp);
    uint16_t* s_ant = reinterpret_cast<uint16_t*>(smem + a.off_ant);

    const ChanInfo ci = a.chans[c];
    const int R = ci.R, W = ci.W, cellsN = R * W;
    const int AP = a.A * P;

    const uint32_t* cp = a.cell_ptr + ci.cell_off;
    const uint16_t* ant = a.ent_ant + ci.ent_off;
    const float* wts = a.ent_w + (int64_t)ci.ent_off * 2 * P;
    if constexpr (CSR_LDS) {
        // one (re, im) pair per pol per entry: float4 for dual pol (16-byte
        // aligned since entry offsets are whole entries), float2 for single pol
        if constexpr (P == 2) {
            const float4* src = reinterpret_cast<const float4*>(wts);
            float4* dst = reinterpret_cast<float4*>(s_w);
            for (int k = tid; k < ci.n_ent; k += THREADS) dst[k] = src[k];
        } else {
            const float2* src = reinterpret_cast<const float2*>(wts);
            float2* dst = reinterpret_cast<float2*>(s_w);
            for (int k = tid; k < ci.n_ent; k += THREADS) dst[k] = src[k];
        }
        for (int k = tid; k <= cellsN; k += THREADS) s_cp[k] = cp[k];
        for (int k = tid; k < ci.n_ent; k += THREADS) s_ant[k] = ant[k];
    }

    // per-lane transform constants
    const bool lane_on = tid < LANES;
    const int q = lane_on ? tid / NK : 0;
    const int kk = lane_on ? tid - q * NK : 0;
    float2 tw[16], wq[Q];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) tw[n1] = a.twiddle[(n1 * q) % N];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) wq[n2] = a.twiddle[(16 * n2 * q) % N];

    float acc[16][NPP];
#pragma unroll
    for (int m = 0; m < 16; ++m)
#pragma unroll
        for (int k = 0; k < NPP; ++k) acc[m][k] = 0.f;

    const bool words = ((AP & 3) == 0) && ((reinterpret_cast<uintptr_t>(a.samples) & 3) == 0);

    for (int64_t t = t0; t < t1; ++t) {
        // 1. decode the (t, c) row of A*P bytes
        const uint8_t* row = a.samples + ((int64_t)t * a.C + c) * AP;
        if (words) {
            const uint32_t* row4 = reinterpret_cast<const uint32_t*>(row);
            for (int w = tid; w < (AP >> 2); w += THREADS) {
                const uint32_t v = row4[w];
                s_smp[4 * w + 0] = unpack44(v & 0xFFu, a.nibble_order);
                s_smp[4 * w + 1] = unpack44((v >> 8) & 0xFFu, a.nibble_order);
                s_smp[4 * w + 2] = unpack44((v >> 16) & 0xFFu, a.nibble_order);
                s_smp[4 * w + 3] = unpack44(v >> 24, a.nibble_order);
            }
        } else {
            for (int k = tid; k < AP; k += THREADS) s_smp[k] = unpack44(row[k], a.nibble_order);
        }
        __syncthreads();

        // 2. gather gridding of the R x W window, both pols per cell
        for (int cell = tid; cell < cellsN; cell += THREADS) {
            const int r = cell / W, w = cell - r * W;
            uint32_t e0, e1;
            if constexpr (CSR_LDS) { e0 = s_cp[cell]; e1 = s_cp[cell + 1]; }
            else { e0 = cp[cell]; e1 = cp[cell + 1]; }
            float2 gx = make_float2(0.f, 0.f), gy = make_float2(0.f, 0.f);
            for (uint32_t e = e0; e < e1; ++e) {
                int an;
                if constexpr (CSR_LDS) an = s_ant[e]; else an = ant[e];
                if constexpr (P == 2) {
                    float4 wt;
                    if constexpr (CSR_LDS) wt = reinterpret_cast<const float4*>(s_w)[e];
                    else wt = reinterpret_cast<const float4*>(wts)[e];
                    const float4 sv = reinterpret_cast<const float4*>(s_smp)[an];
                    gx = cfma(gx, make_float2(wt.x, wt.y), make_float2(sv.x, sv.y));
                    gy = cfma(gy, make_float2(wt.z, wt.w), make_float2(sv.z, sv.w));
                } else {
                    float2 wt;
                    if constexpr (CSR_LDS) wt = reinterpret_cast<const float2*>(s_w)[e];
                    else wt = reinterpret_cast<const float2*>(wts)[e];
                    gx = cfma(gx, wt, s_smp[an]);
                }
            }
            s_G[r * a.WP + w] = gx;
            if constexpr (P == 2) s_G[(a.Rmax + r) * a.WP + w] = gy;
        }
        __syncthreads();

        // 3a. row pass: R rows per pol, outputs for this workgroup's columns
        if (lane_on) {
            for (int rr = kk; rr < P * R; rr += NK) {
                const int p = (P == 2 && rr >= R) ? 1 : 0;
                const int r = rr - p * R;
                float2 z[16];
                fold_twiddle<Q>(z, s_G + (p * a.Rmax + r) * a.WP, 1, W, tw, wq);
                fft16(z);
                float2* yrow = s_Y + (p * a.Rmax + r) * a.YP;
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    if ((m / (16 / KS)) == kpart) yrow[q + Q * m - kpart * NK] = z[fft16_pos(m)];
                }
            }
        }
        __syncthreads();

        // 3b + 4. column pass per pol, products and accumulation in registers
        if (lane_on) {
            float2 X[16];
            fold_twiddle<Q>(X, s_Y + kk, a.YP, R, tw, wq);
            fft16(X);
            if constexpr (P == 2) {
                float2 Yv[16];
                fold_twiddle<Q>(Yv, s_Y + a.Rmax * a.YP + kk, a.YP, R, tw, wq);
                fft16(Yv);
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const float2 x = X[fft16_pos(m)], y = Yv[fft16_pos(m)];
                    acc[m][0] = fmaf(x.x, x.x, fmaf(x.y, x.y, acc[m][0]));
                    acc[m][1] = fmaf(y.x, y.x, fmaf(y.y, y.y, acc[m][1]));
                    acc[m][2] = fmaf(x.x, y.x, fmaf(x.y, y.y, acc[m][2]));
                    acc[m][3] = fmaf(x.y, y.x, fmaf(-x.x, y.y, acc[m][3]));
                }
            } else {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const float2 x = X[fft16_pos(m)];
                    acc[m][0] = fmaf(x.x, x.x, fmaf(x.y, x.y, acc[m][0]));
                }
            }
        }
        // the next iteration's first barrier orders these LDS reads before the
        // next row pass overwrites s_Y
    }

    // add this work item's sums into its slot; bin (k', j') -> pixel (k'+N/2, j'+N/2) mod N
    if (lane_on) {
        const int kb = kpart * NK + kk;
        int i = kb + N / 2;
        if (i >= N) i -= N;
        float* base = a.slots + ((int64_t)s * a.C + c) * NPP * N * N;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            int j = q + Q * m + N / 2;
            if (j >= N) j -= N;
#pragma unroll
            for (int k = 0; k < NPP; ++k) {
                float* dst = base + ((int64_t)k * N + j) * N + i;
                *dst += acc[m][k];
            }
        }
    }
}

struct Layout {
    uint32_t off_w, off_smp, off_G, off_Y, off_cp, off_ant;
    size_t total;
    int WP, YP;
};

Layout layout(const SubDev& d, int KS, bool csr_lds) {
    Layout L{};
    size_t b = 0;
    auto take = [&](size_t n) {
        b = (b + 15) & ~(size_t)15;
        size_t o = b;
        b += n;
        return (uint32_t)o;
    };
    L.WP = d.Wmax | 1;                 // odd row pitch (float2) against LDS bank conflicts
    L.YP = d.N / KS + 1;
    L.off_w = csr_lds ? take((size_t)d.Emax * 2 * d.P * sizeof(float)) : 0;
    L.off_smp = take((size_t)d.A * d.P * sizeof(float2));
    L.off_G = take((size_t)d.P * d.Rmax * L.WP * sizeof(float2));
    L.off_Y = take((size_t)d.P * d.Rmax * L.YP * sizeof(float2));
    L.off_cp = csr_lds ? take(((size_t)d.Rmax * d.Wmax + 1) * sizeof(uint32_t)) : 0;
    L.off_ant = csr_lds ? take((size_t)d.Emax * sizeof(uint16_t)) : 0;
    L.total = (b + 15) & ~(size_t)15;
    return L;
}

using KernelFn = void (*)(Fp32Args);

template <int Q, int P>
KernelFn pick(bool csr) {
    return csr ? fp32_kernel<Q, P, true> : fp32_kernel<Q, P, false>;
}

KernelFn select_kernel(int Q, int P, bool csr) {
    switch (Q * 2 + (P - 1)) {
#define EPIC_CASE(QQ)                             \
    case QQ * 2 + 0: return pick<QQ, 1>(csr);     \
    case QQ * 2 + 1: return pick<QQ, 2>(csr);
        EPIC_CASE(1) EPIC_CASE(2) EPIC_CASE(3) EPIC_CASE(4) EPIC_CASE(5) EPIC_CASE(6) EPIC_CASE(7) EPIC_CASE(8)
#undef EPIC_CASE
    }
    return nullptr;
}

int threads_for(int Q) {
    switch (Q) {
        case 1: return Shape<1>::THREADS;
        case 2: return Shape<2>::THREADS;
        case 3: return Shape<3>::THREADS;
        case 4: return Shape<4>::THREADS;
        case 5: return Shape<5>::THREADS;
        case 6: return Shape<6>::THREADS;
        case 7: return Shape<7>::THREADS;
        case 8: return Shape<8>::THREADS;
    }
    return 0;
}

constexpr size_t kLdsLimit = 160 * 1024;

}  // namespace

// Choose the launch shape (pure host arithmetic).  The gather lists live in LDS
// when they fit next to the per-spectrum buffers, else they stream from L2.
// device < 0: no HIP calls (dry run).
hipError_t fp32_configure(SubDev& d, int device) {
    const int Q = d.N / 16;
    if (Q < 1 || Q > 8 || d.N % 16 != 0) return hipErrorNotSupported;
    d.KS = (Q >= 7) ? 2 : 1;
    d.threads = threads_for(Q);
    Layout with = layout(d, d.KS, true);
    Layout without = layout(d, d.KS, false);
    d.csr_in_lds = (with.total <= kLdsLimit / 2 || (with.total <= kLdsLimit && without.total > kLdsLimit / 2)) ? 1 : 0;
    const Layout& L = d.csr_in_lds ? with : without;
    if (L.total > kLdsLimit) return hipErrorNotSupported;
    d.lds_bytes = L.total;
    if (device >= 0) {
        KernelFn fn = select_kernel(Q, d.P, d.csr_in_lds != 0);
        if (!fn) return hipErrorNotSupported;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fp32(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st) {
    const int Q = d.N / 16;
    const Layout L = layout(d, d.KS, d.csr_in_lds != 0);
    Fp32Args a{};
    a.samples = samples;
    a.T = n_time;
    a.C = d.C; a.A = d.A; a.S = d.S;
    a.chans = d.chans; a.cell_ptr = d.cell_ptr; a.ent_ant = d.ent_ant; a.ent_w = d.ent_w;
    a.twiddle = d.twiddle; a.slots = d.slots;
    a.Rmax = d.Rmax; a.WP = L.WP; a.YP = L.YP;
    a.off_w = L.off_w; a.off_smp = L.off_smp; a.off_G = L.off_G; a.off_Y = L.off_Y;
    a.off_cp = L.off_cp; a.off_ant = L.off_ant;
    a.nibble_order = d.nibble_order;
    a.units = d.C * d.S * d.KS;
    a.units_per_xcd = (a.units + 7) / 8;
    KernelFn fn = select_kernel(Q, d.P, d.csr_in_lds != 0);
    if (!fn) return hipErrorNotSupported;
    hipLaunchKernelGGL(fn, dim3(8 * a.units_per_xcd), dim3(d.threads), L.total, st, a);
    return hipGetLastError();
}

}  // namespace epic
