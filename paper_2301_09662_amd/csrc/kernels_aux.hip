// One-off FP64 set-up kernels (kernel taps, transform tables, gather-entry
// weights), the ordered read-out of the partial accumulators, and the debug
// decoder.  FP64 appears only here, never on the per-spectrum path.
#include "epic_internal.hpp"
#include "epic_device.hpp"

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
// Layout per entry: real taps -> P floats (re per pol); complex -> 2P floats.
// One thread per entry slot of one channel.
__global__ void entry_weights_kernel(const ChanInfo* __restrict__ chans, const uint16_t* __restrict__ grp_ant,
                                     const uint8_t* __restrict__ grp_tap, const float* __restrict__ taps,
                                     const float* __restrict__ gains, float* __restrict__ grp_w, int C, int A,
                                     int P, int K, int real) {
    const int c = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const ChanInfo ci = chans[c];
    if (e >= ci.n_grp * kGroup) return;
    const int64_t ge = (int64_t)ci.grp_off * kGroup + e;
    const int a = grp_ant[ge], tap = grp_tap[ge];
    const int wf = real ? P : 2 * P;
    for (int p = 0; p < P; ++p) {
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
        if (real) {
            grp_w[ge * wf + p] = (float)wr;
        } else {
            grp_w[ge * wf + 2 * p + 0] = (float)wr;
            grp_w[ge * wf + 2 * p + 1] = (float)wi;
        }
    }
}

// out[c][k][j][i] = sum_s slots[s][c][k][j][i], summed in slot order so the
// result is identical from run to run; Stokes form on request (linear feeds:
// I = XX+YY, Q = XX-YY, U = 2 Re XY*, V = -2 Im XY*); optional reset.
__global__ void readout_kernel(float* __restrict__ slots, float* __restrict__ out, int S, int C, int NPP,
                               int NN, int stokes, int reset) {
    const int64_t per_slot = (int64_t)C * NPP * NN;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over C * NN pixels
    if (idx >= (int64_t)C * NN) return;
    const int64_t c = idx / NN, pix = idx - c * NN;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < NPP; ++k) v[k] += slots[s * per_slot + (c * NPP + k) * NN + pix];
    if (stokes && NPP == 4) {
        const float I = v[0] + v[1], Q = v[0] - v[1], U = 2.0f * v[2], V = -2.0f * v[3];
        v[0] = I; v[1] = Q; v[2] = U; v[3] = V;
    }
    for (int k = 0; k < NPP; ++k) out[(c * NPP + k) * NN + pix] = v[k];
    if (reset)
        for (int s = 0; s < S; ++s)
            for (int k = 0; k < NPP; ++k) slots[s * per_slot + (c * NPP + k) * NN + pix] = 0.0f;
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
        d.chans, d.grp_ant, d.grp_tap, d.taps, d.gains, d.grp_w, d.C, d.A, d.P, d.K, d.real_taps);
    return hipGetLastError();
}

hipError_t launch_readout(const SubDev& d, float* out, int stokes, int reset, hipStream_t st) {
    const int64_t n = (int64_t)d.C * d.N * d.N;
    const int bs = 256;
    readout_kernel<<<dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st>>>(d.slots, out, d.S, d.C, d.NPP, d.N * d.N,
                                                                            stokes, reset);
    return hipGetLastError();
}

hipError_t launch_unpack_debug(const uint8_t* in, int64_t n, int order, float* out, hipStream_t st) {
    const int bs = 256;
    unpack_debug_kernel<<<dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st>>>(in, n, order,
                                                                                 reinterpret_cast<float2*>(out));
    return hipGetLastError();
}

}  // namespace epic
