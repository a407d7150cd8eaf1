// One-off FP64 set-up kernels (kernel taps, transform tables, gather-entry
// weights), the zero-lag correlations and ordered read-out of the partial
// accumulators, and the debug decoder.  FP64 appears only in the set-up
// kernels, never on the per-spectrum or per-integration path.
#include "epic_internal.hpp"
#include "epic_device.hpp"
#include "epic_gather.hpp"

namespace epic {

namespace {

// Default gridding kernel: a K x K Gaussian of the distance between each tap's
// cell centre and the antenna's fractional position g, normalised to unit sum
// (nearest-cell kernels of Sec. 3.1; the shape is this library's choice).
// One thread per (channel, antenna); the same kernel is used for every pol.
__global__ void gaussian_taps_kernel(const int32_t* __restrict__ cells, const double* __restrict__ g,
                                     float* __restrict__ taps, int C, int A, int P, int K, double sigma) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)C * A) return;
    const int h = K / 2;
    const double cx = (double)cells[2 * idx], cy = (double)cells[2 * idx + 1];
    const double gx = g[2 * idx], gy = g[2 * idx + 1];
    const double inv = 1.0 / (2.0 * sigma * sigma);
    double w[49];
    double sum = 0.0;
    for (int dy = -h; dy <= h; ++dy)
        for (int dx = -h; dx <= h; ++dx) {
            const double ex = cx + dx - gx, ey = cy + dy - gy;
            const double v = exp(-(ex * ex + ey * ey) * inv);
            w[(dy + h) * K + (dx + h)] = v;
            sum += v;
        }
    float* out = taps + idx * (int64_t)P * K * K * 2;
    for (int p = 0; p < P; ++p)
        for (int k = 0; k < K * K; ++k) {
            out[(p * K * K + k) * 2 + 0] = (float)(w[k] / sum);
            out[(p * K * K + k) * 2 + 1] = 0.0f;
        }
}

// exp(+2 pi i r / N), r = 0..N-1, evaluated in FP64 and rounded once.
__global__ void twiddle_kernel(float2* __restrict__ tw, int N) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double s, c;
    sincospi(2.0 * (double)r / (double)N, &s, &c);
    tw[r] = make_float2((float)c, (float)s);
}

// Weight of every gather entry: the entry's tap times the antenna's gain,
// complex product in FP64, rounded once.  Padding entries (tap 255) weigh 0.
// Layout per entry by weight mode: complex -> 2P floats (re, im per pol);
// real -> P floats (re per pol); shared -> 1 float (the X weight, equal to Y).
// One thread per entry slot of one channel.
__global__ void entry_weights_kernel(const ChanInfo* __restrict__ chans, const uint16_t* __restrict__ grp_ant,
                                     const uint8_t* __restrict__ grp_tap, const float* __restrict__ taps,
                                     const float* __restrict__ gains, float* __restrict__ grp_w, int C, int A,
                                     int P, int K, int wm) {
    const int c = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const ChanInfo ci = chans[c];
    if (e >= ci.n_grp * kGroup) return;
    const int64_t ge = (int64_t)ci.grp_off * kGroup + e;
    const int a = grp_ant[ge], tap = grp_tap[ge];
    const int wf = wm == kWComplex ? 2 * P : (wm == kWReal ? P : 1);
    for (int p = 0; p < (wm == kWShared ? 1 : P); ++p) {
        double wr = 0.0, wi = 0.0;
        if (tap != 255) {
            const int64_t ti = ((((int64_t)c * A + a) * P + p) * K * K + tap) * 2;
            wr = taps[ti];
            wi = taps[ti + 1];
            if (gains) {
                const int64_t gi = (((int64_t)c * A + a) * P + p) * 2;
                const double gr = gains[gi], gim = gains[gi + 1];
                const double r = gr * wr - gim * wi, i = gr * wi + gim * wr;
                wr = r;
                wi = i;
            }
        }
        if (wm != kWComplex) {
            grp_w[ge * wf + p] = (float)wr;
        } else {
            grp_w[ge * wf + 2 * p + 0] = (float)wr;
            grp_w[ge * wf + 2 * p + 1] = (float)wi;
        }
    }
}

// ---- autocorrelations (the a = b terms of Eq. 3) ---------------------------
// Zero-lag correlations of every antenna over the spectra of a call:
// vaa[c][a] += (XX*, YY*, Re XY*, Im XY*) (single pol: XX* only).  One thread
// per (channel, antenna) sums kAutoChunk spectra in registers and adds them
// with one integer atomic per product.  Every term is an integer of magnitude
// at most 128 (products of 4-bit numbers), so the int32 sums are exact and
// independent of the order of the atomics up to 2^24 - 1 spectra; the host
// folds them into the lag sums before a call would pass that count.
constexpr int kAutoChunk = 64;

__device__ __forceinline__ int2 unpack44_int(uint32_t byte, int order) {
    const int hi = ((int)(byte << 24)) >> 28;
    const int lo = ((int)(byte << 28)) >> 28;
    return order == 0 ? make_int2(hi, lo) : make_int2(lo, hi);
}

__global__ void autocorr_accumulate_kernel(const uint8_t* __restrict__ samples, int64_t T, int C, int A, int P,
                                           int nibble_order, int32_t* __restrict__ vaa) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // c * A + a
    if (idx >= (int64_t)C * A) return;
    const int64_t c = idx / A, a = idx - c * A;
    const int64_t t0 = (int64_t)blockIdx.y * kAutoChunk;
    const int64_t t1 = (t0 + kAutoChunk < T) ? t0 + kAutoChunk : T;
    const int64_t AP = (int64_t)A * P;
    int xx = 0, yy = 0, xyr = 0, xyi = 0;
    for (int64_t t = t0; t < t1; ++t) {
        const uint8_t* row = samples + (t * C + c) * AP + a * P;
        const int2 x = unpack44_int(row[0], nibble_order);
        xx += x.x * x.x + x.y * x.y;
        if (P == 2) {
            const int2 y = unpack44_int(row[1], nibble_order);
            yy += y.x * y.x + y.y * y.y;
            xyr += x.x * y.x + x.y * y.y;
            xyi += x.y * y.x - x.x * y.y;
        }
    }
    const int npa = (P == 2) ? 4 : 1;
    int32_t* dst = vaa + idx * npa;
    atomicAdd(dst, xx);
    if (P == 2) {
        atomicAdd(dst + 1, yy);
        atomicAdd(dst + 2, xyr);
        atomicAdd(dst + 3, xyi);
    }
}

// Lag sums of one channel: R^{pq}(d) = sum_a V^{pq}_aa sum_u w^p_a(u + d) conj(w^q_a(u))
// for every tap offset d in [-(K-1), K-1]^2 (the correlation of the antenna's
// kernel with itself, weighted by its zero-lag correlation).  An antenna's
// kernel image times its conjugate depends on these lags only, not on where
// the antenna sits, so sum_d R(d) exp(+2 pi i d.k / N) is the image of the
// a = b terms.  Products: 0 XX* (w^X, w^X), 1 YY* (w^Y, w^Y), 2 XY* (w^X, w^Y).
// Block (lag, channel); threads stride over antennas; FP32 sums in a fixed
// order, added into the lag accumulator (which thus holds the a = b terms of
// several stretches of an integration with different gains).
// lag layout: [C][L][npl][2] with L = (2K-1)^2, npl = 3 (dual pol) or 1.
__global__ void autocorr_lag_kernel(const int32_t* __restrict__ vaa, const float* __restrict__ taps,
                                    const float* __restrict__ gains, float* __restrict__ lag, int C, int A, int P,
                                    int K) {
    const int L1 = 2 * K - 1;
    const int l = blockIdx.x, c = blockIdx.y;
    const int ddy = l / L1 - (K - 1), ddx = l % L1 - (K - 1);
    const int npl = (P == 2) ? 3 : 1, npa = (P == 2) ? 4 : 1;
    float acc[3][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
    for (int a = threadIdx.x; a < A; a += blockDim.x) {
        const int32_t* v = vaa + ((int64_t)c * A + a) * npa;
        for (int q = 0; q < npl; ++q) {
            const int pa = (q == 1) ? 1 : 0, pb = (q == 0) ? 0 : 1;
            float gr[2] = {1.f, 1.f}, gi[2] = {0.f, 0.f};
            if (gains)
                for (int h = 0; h < 2; ++h) {
                    const int p = h ? pb : pa;
                    const int64_t gix = (((int64_t)c * A + a) * P + p) * 2;
                    gr[h] = gains[gix];
                    gi[h] = gains[gix + 1];
                }
            float sr = 0.f, si = 0.f;   // sum_u w^pa(u + d) conj(w^pb(u))
            for (int uy = 0; uy < K; ++uy) {
                const int vy = uy + ddy;
                if (vy < 0 || vy >= K) continue;
                for (int ux = 0; ux < K; ++ux) {
                    const int vx = ux + ddx;
                    if (vx < 0 || vx >= K) continue;
                    const float* ta = taps + ((((int64_t)c * A + a) * P + pa) * K * K + vy * K + vx) * 2;
                    const float* tb = taps + ((((int64_t)c * A + a) * P + pb) * K * K + uy * K + ux) * 2;
                    // gains applied to the taps as the gridding does
                    const float ar = gr[0] * ta[0] - gi[0] * ta[1], ai = gr[0] * ta[1] + gi[0] * ta[0];
                    const float br = gr[1] * tb[0] - gi[1] * tb[1], bi = gr[1] * tb[1] + gi[1] * tb[0];
                    sr += ar * br + ai * bi;
                    si += ai * br - ar * bi;
                }
            }
            float vr, vi;
            if (q == 0) { vr = (float)v[0]; vi = 0.f; }
            else if (q == 1) { vr = (float)v[1]; vi = 0.f; }
            else { vr = (float)v[2]; vi = (float)v[3]; }
            acc[q][0] += vr * sr - vi * si;
            acc[q][1] += vr * si + vi * sr;
        }
    }
    // block reduction (fixed order: deterministic)
    __shared__ float red[256][6];
    for (int q = 0; q < 3; ++q) {
        red[threadIdx.x][2 * q] = acc[q][0];
        red[threadIdx.x][2 * q + 1] = acc[q][1];
    }
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 6; ++k) red[threadIdx.x][k] += red[threadIdx.x + w][k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int L = L1 * L1;
        float* out = lag + (((int64_t)c * L + l) * npl) * 2;
        for (int q = 0; q < npl; ++q) {
            out[2 * q] += red[0][2 * q];
            out[2 * q + 1] += red[0][2 * q + 1];
        }
    }
}

// out[c][k][j][i] = sum_s slots[s][c][k][j][i], summed in slot order so the
// result is identical from run to run; minus the autocorrelation image when
// lag != nullptr; Stokes form on request (linear feeds, XY* = (U + i V) / 2:
// I = XX+YY, Q = XX-YY, U = 2 Re XY*, V = 2 Im XY*); optional reset of the
// slots.  The autocorrelation image at pixel (i, j) reads frequency bin
// k = (i + N/2, j + N/2) mod N, where exp(+2 pi i d.k / N) =
// (-1)^(dx+dy) exp(+2 pi i (dx i + dy j) / N), the phase from the plan's table
// tw[r] = exp(+2 pi i r / N) (FP64 at plan time, rounded once to FP32).
__global__ void readout_kernel(float* __restrict__ slots, float* __restrict__ out, int S, int C, int NPP,
                               int N, int stokes, int reset, const float* __restrict__ lag, int K,
                               const float2* __restrict__ tw) {
    const int NN = N * N;
    const int64_t per_slot = (int64_t)C * NPP * NN;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over C * NN pixels
    if (idx >= (int64_t)C * NN) return;
    const int64_t c = idx / NN, pix = idx - c * NN;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < NPP; ++k) v[k] += slots[s * per_slot + (c * NPP + k) * NN + pix];
    if (lag) {
        const int i = (int)(pix % N), j = (int)(pix / N);
        const int L1 = 2 * K - 1, npl = (NPP == 4) ? 3 : 1;
        const float* lc = lag + (int64_t)c * L1 * L1 * npl * 2;
        float ar[3] = {0.f, 0.f, 0.f}, ai[3] = {0.f, 0.f, 0.f};
        for (int l = 0; l < L1 * L1; ++l) {
            const int dy = l / L1 - (K - 1), dx = l % L1 - (K - 1);
            int r = (dx * i + dy * j) % N;
            if (r < 0) r += N;
            const float2 ph = tw[r];
            const float sg = ((dx + dy) & 1) ? -1.f : 1.f;
            const float er = sg * ph.x, ei = sg * ph.y;
            for (int q = 0; q < npl; ++q) {
                const float lr = lc[(l * npl + q) * 2], li = lc[(l * npl + q) * 2 + 1];
                ar[q] = fmaf(lr, er, fmaf(-li, ei, ar[q]));
                ai[q] = fmaf(lr, ei, fmaf(li, er, ai[q]));
            }
        }
        v[0] -= ar[0];
        if (NPP == 4) {
            v[1] -= ar[1];
            v[2] -= ar[2];
            v[3] -= ai[2];
        }
    }
    if (stokes && NPP == 4) {
        const float I = v[0] + v[1], Q = v[0] - v[1], U = 2.0f * v[2], V = 2.0f * v[3];
        v[0] = I; v[1] = Q; v[2] = U; v[3] = V;
    }
    for (int k = 0; k < NPP; ++k) out[(c * NPP + k) * NN + pix] = v[k];
    if (reset)
        for (int s = 0; s < S; ++s)
            for (int k = 0; k < NPP; ++k) slots[s * per_slot + (c * NPP + k) * NN + pix] = 0.0f;
}

__global__ void zero_kernel(float* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0f;
}

__global__ void unpack_debug_kernel(const uint8_t* __restrict__ in, int64_t n, int order, float2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = unpack44(in[i], order);
}

}  // namespace

hipError_t launch_gaussian_taps(const SubDev& d, double sigma, hipStream_t st) {
    const int64_t n = (int64_t)d.C * d.A;
    const int bs = 128;
    gaussian_taps_kernel<<<dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st>>>(d.cells, d.gfrac, d.taps, d.C, d.A,
                                                                                   d.P, d.K, sigma);
    return hipGetLastError();
}

hipError_t launch_twiddles(const SubDev& d, hipStream_t st) {
    twiddle_kernel<<<dim3((d.N + 63) / 64), dim3(64), 0, st>>>(d.twiddle, d.N);
    return hipGetLastError();
}

hipError_t launch_entry_weights(const SubDev& d, hipStream_t st) {
    const int bs = 256;
    entry_weights_kernel<<<dim3((d.Gmax * kGroup + bs - 1) / bs, d.C), dim3(bs), 0, st>>>(
        d.chans, d.grp_ant, d.grp_tap, d.taps, d.gains, d.grp_w, d.C, d.A, d.P, d.K, d.wmode);
    return hipGetLastError();
}

hipError_t launch_autocorr(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st) {
    const int64_t n = (int64_t)d.C * d.A;
    const int bs = 256;
    const int64_t chunks = (n_time + kAutoChunk - 1) / kAutoChunk;
    if (chunks > 65535) return hipErrorInvalidValue;
    autocorr_accumulate_kernel<<<dim3((unsigned)((n + bs - 1) / bs), (unsigned)chunks), dim3(bs), 0, st>>>(
        samples, n_time, d.C, d.A, d.P, d.nibble_order, d.vaa);
    return hipGetLastError();
}

hipError_t launch_zero(float* x, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    zero_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(x, n);
    return hipGetLastError();
}

int64_t vaa_count(const SubDev& d) { return (int64_t)d.C * d.A * (d.P == 2 ? 4 : 1); }
int64_t lag_count(const SubDev& d) { return (int64_t)d.C * (2 * d.K - 1) * (2 * d.K - 1) * (d.P == 2 ? 3 : 1) * 2; }

// Move the zero-lag correlations gathered so far into the lag accumulator
// (with the gains in effect while they were gathered) and clear them.
hipError_t launch_autocorr_fold(const SubDev& d, hipStream_t st) {
    if (!d.vaa) return hipSuccess;
    const int L1 = 2 * d.K - 1;
    autocorr_lag_kernel<<<dim3(L1 * L1, d.C), dim3(256), 0, st>>>(d.vaa, d.taps, d.gains, d.lag, d.C, d.A, d.P, d.K);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_zero(reinterpret_cast<float*>(d.vaa), vaa_count(d), st);   // all-zero bits: 0 as int32 too
}

hipError_t launch_readout(const SubDev& d, float* out, int stokes, int reset, hipStream_t st) {
    const int64_t n = (int64_t)d.C * d.N * d.N;
    const int bs = 256;
    hipError_t e = launch_autocorr_fold(d, st);
    if (e != hipSuccess) return e;
    readout_kernel<<<dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st>>>(
        d.slots, out, d.S, d.C, d.NPP, d.N, stokes, reset, d.vaa ? d.lag : nullptr, d.K, d.twiddle);
    e = hipGetLastError();
    if (e != hipSuccess || !reset || !d.vaa) return e;
    return launch_zero(d.lag, lag_count(d), st);
}

hipError_t launch_unpack_debug(const uint8_t* in, int64_t n, int order, float* out, hipStream_t st) {
    const int bs = 256;
    unpack_debug_kernel<<<dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st>>>(in, n, order,
                                                                                 reinterpret_cast<float2*>(out));
    return hipGetLastError();
}

}  // namespace epic
