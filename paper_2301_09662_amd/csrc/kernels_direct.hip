// Direct imaging on the matrix cores (EPIC_GRID_DIRECT_GEMM): no aperture grid
// and no FFT.  Gridding and the inverse transform of Eq. 4 are both linear, so
// their composition is one matrix per channel: the field of pixel q is
//   E~_q = sum_a M_c[q][a] E_a,   M_c[q][a] = sum over antenna a's taps of
//          w (-1)^(x+y) exp(+2 pi i (x i + y j) / N)            (q = (j, i))
// -- each antenna's kernel image.  The work is O(A N^2) per spectrum against
// O(N^2 log N) for grid + FFT, which the paper's argument for the FFT route
// favours at scale (Sec. 1); for small arrays on small grids the product is
// cheap on the matrix cores and needs neither the gather nor two transform
// passes.  It runs in real form on 16 x 16 x 32 FP16 MFMA:
//   rows     8 pixels x (re, im) of the output field;
//   depth    16 antennas x (re, im) of the input field;
//   columns  the spectra of a step x the pols (8 x 2 or 16 x 1).
// M is split into FP16 high + low parts (products summed in FP32), built once
// in FP64 from the taps and gains.  A workgroup owns a channel, a range of
// pixel tiles (whose M fragments it keeps in registers for the whole call) and
// a stretch of spectra; the products of Eq. 5 are formed by exchanging the X
// and Y fields between neighbouring lanes and are summed over the spectra in
// registers, then into the stretch's partial-accumulator slot.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "epic_device.hpp"
#include "epic_gather.hpp"
#include "epic_internal.hpp"
#include "epic_mfma.hpp"

namespace epic {

namespace {

constexpr int kDirWaves = 4;       // waves per workgroup
constexpr int kDirTilesPerWave = 2;   // 8-pixel tiles per wave
constexpr int kDirMaxBlk = 4;      // antenna blocks of 16 (A <= 64)

struct DirArgs {
    const uint8_t* samples;   // [T][C][A][P]
    const half8* m;           // [C][tiles][blk][2 terms][64 lanes] A-operand fragments
    float* slots;             // [S][C][NPP][N][N]
    int64_t T;
    int C, A, N, nblk, ntile, groups, chunks, nibble_order;
    int fresh;                // 1: the slots hold zeros, store instead of add
    uint32_t off_E;           // LDS: two buffers of [blk][64 lanes] half8
};

template <int P, int NBLK>
__global__ void __launch_bounds__(64 * kDirWaves) direct_kernel(DirArgs a) {
    constexpr int TB = 16 / P;   // spectra per step: 16 columns = TB spectra x P pols
    constexpr int NPP = (P == 2) ? 4 : 1;
    const int wg = blockIdx.x;
    const int chunk = wg % a.chunks;
    const int grp = (wg / a.chunks) % a.groups;
    const int c = wg / (a.chunks * a.groups);
    if (c >= a.C) return;
    // this workgroup's stretch of spectra [t0, t1): its chunk of the call
    const int64_t t0 = a.T * chunk / a.chunks, t1 = a.T * (chunk + 1) / a.chunks;
    if (t0 >= t1) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, l4 = lane >> 4;
    extern __shared__ __align__(16) unsigned char smem[];
    half8* s_E = reinterpret_cast<half8*>(smem + a.off_E);

    // the wave's pixel tiles and their M fragments (kept for the whole call)
    int tile[kDirTilesPerWave];
    half8 mh[kDirTilesPerWave][NBLK], ml[kDirTilesPerWave][NBLK];
#pragma unroll
    for (int k = 0; k < kDirTilesPerWave; ++k) {
        tile[k] = (grp * kDirWaves + wave) * kDirTilesPerWave + k;
        const bool on = tile[k] < a.ntile;
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            const size_t o = ((((size_t)c * a.ntile + (on ? tile[k] : 0)) * NBLK + b) * 2) * 64 + lane;
            mh[k][b] = a.m[o];
            ml[k][b] = a.m[o + 64];
        }
    }
    float acc[kDirTilesPerWave][4];
#pragma unroll
    for (int k = 0; k < kDirTilesPerWave; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[k][e] = 0.f;

    // decode the step's spectra into the field operand: element (antenna a,
    // re/im r) of block a / 16 is row k = 2 (a % 16) + r, column n = u P + p,
    // held by lane 16 (k / 8) + n at position k % 8
    auto decode = [&](half8* dst, int64_t tb, int nb) {
        _Float16* d16 = reinterpret_cast<_Float16*>(dst);
        for (int task = tid; task < TB * NBLK * 16; task += 64 * kDirWaves) {
            const int u = task / (NBLK * 16);
            const int an = task - u * NBLK * 16;
            const int b = an >> 4, ai = an & 15;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                float2 v = make_float2(0.f, 0.f);
                if (u < nb && an < a.A)
                    v = unpack44(a.samples[((tb + u) * a.C + c) * (int64_t)a.A * P + (int64_t)an * P + p],
                                 a.nibble_order);
                const int n = u * P + p;
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int k = 2 * ai + r;
                    d16[((b * 64) + 16 * (k >> 3) + n) * 8 + (k & 7)] = (_Float16)(r ? v.y : v.x);
                }
            }
        }
    };

    int buf = 0;
    decode(s_E, t0, (int)std::min<int64_t>(TB, t1 - t0));
    __syncthreads();
    for (int64_t tb = t0; tb < t1; tb += TB) {
        const int64_t nxt = tb + TB;
        // the next step's fields into the other buffer while this one multiplies
        if (nxt < t1) decode(s_E + (buf ^ 1) * NBLK * 64, nxt, (int)std::min<int64_t>(TB, t1 - nxt));
        half8 eb[NBLK];
#pragma unroll
        for (int b = 0; b < NBLK; ++b) eb[b] = s_E[(buf * NBLK + b) * 64 + lane];
#pragma unroll
        for (int k = 0; k < kDirTilesPerWave; ++k) {
            floatx4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                d = mfma16(mh[k][b], eb[b], d);
                d = mfma16(ml[k][b], eb[b], d);
            }
            // lane: pixels 2 l4 and 2 l4 + 1 of the tile (re, im each), column l16;
            // columns beyond the step's spectra hold zero fields
            if constexpr (P == 2) {
                // X (even column) and Y (odd column) of one spectrum in neighbouring lanes
                floatx4 o;
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = __shfl_xor(d[e], 1);
                const bool xl = (l16 & 1) == 0;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float xr = xl ? d[2 * s] : o[2 * s], xi = xl ? d[2 * s + 1] : o[2 * s + 1];
                    const float yr = xl ? o[2 * s] : d[2 * s], yi = xl ? o[2 * s + 1] : d[2 * s + 1];
                    // even lane: XX*, Re XY*; odd lane: YY*, Im XY*
                    const float own_r = xl ? xr : yr, own_i = xl ? xi : yi;
                    acc[k][2 * s] = fmaf(own_r, own_r, fmaf(own_i, own_i, acc[k][2 * s]));
                    acc[k][2 * s + 1] = xl ? fmaf(xr, yr, fmaf(xi, yi, acc[k][2 * s + 1]))
                                           : fmaf(xi, yr, fmaf(-xr, yi, acc[k][2 * s + 1]));
                }
            } else {
#pragma unroll
                for (int s = 0; s < 2; ++s) acc[k][s] = fmaf(d[2 * s], d[2 * s], fmaf(d[2 * s + 1], d[2 * s + 1], acc[k][s]));
            }
        }
        __syncthreads();   // every wave is done with this buffer; the next one is written
        buf ^= 1;
    }

    // sum over the step's columns (spectra): lanes of one pixel pair and pol
#pragma unroll
    for (int k = 0; k < kDirTilesPerWave; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float v = acc[k][e];
            for (int m = P; m < 16; m <<= 1) v += __shfl_xor(v, m);
            acc[k][e] = v;
        }
    const int N = a.N, NN = N * N;
    float* out = a.slots + ((int64_t)chunk * a.C + c) * NPP * NN;
#pragma unroll
    for (int k = 0; k < kDirTilesPerWave; ++k) {
        if (tile[k] >= a.ntile || l16 >= P) continue;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int q = tile[k] * 8 + 2 * l4 + s;   // pixel j * N + i
            if constexpr (P == 2) {
                const int pa = l16 == 0 ? 0 : 1, pb = l16 == 0 ? 2 : 3;   // XX*, Re XY* / YY*, Im XY*
                slot_put(&out[(int64_t)pa * NN + q], acc[k][2 * s], a.fresh != 0);
                slot_put(&out[(int64_t)pb * NN + q], acc[k][2 * s + 1], a.fresh != 0);
            } else {
                slot_put(&out[q], acc[k][s], a.fresh != 0);
            }
        }
    }
}

// M in FP64: thread per (channel, pixel, antenna); the A-operand fragment
// element of (pixel row (q, r_out), antenna column (a, r_in)) of the real form
// [[Mr, -Mi], [Mi, Mr]], split into FP16 hi and lo.
__global__ void direct_matrix_kernel(const int32_t* __restrict__ cells, const float* __restrict__ taps,
                                     const float* __restrict__ gains, half8* __restrict__ m, int C, int A, int P,
                                     int K, int N, int nblk) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int NN = N * N;
    if (idx >= (int64_t)C * NN * nblk * 16) return;
    const int an = (int)(idx % (nblk * 16));
    const int64_t cq = idx / (nblk * 16);
    const int q = (int)(cq % NN), c = (int)(cq / NN);
    double mr = 0.0, mi = 0.0;
    if (an < A) {
        const int h = K / 2;
        const int64_t ca = (int64_t)c * A + an;
        const int cx = cells[2 * ca], cy = cells[2 * ca + 1];
        const int i = q % N, j = q / N;
        double gr = 1.0, gi = 0.0;
        if (gains) {
            gr = gains[ca * P * 2];
            gi = gains[ca * P * 2 + 1];
        }
        for (int dy = -h; dy <= h; ++dy)
            for (int dx = -h; dx <= h; ++dx) {
                const int x = cx + dx, y = cy + dy;
                const float* t = taps + (ca * P * K * K + (dy + h) * K + (dx + h)) * 2;   // pol 0 (shared)
                const double wr = gr * t[0] - gi * t[1], wi = gr * t[1] + gi * t[0];
                const int r = (int)(((int64_t)x * i + (int64_t)y * j) % N);
                double s, co;
                sincospi(2.0 * (double)r / (double)N, &s, &co);
                const double sg = ((x + y) & 1) ? -1.0 : 1.0;
                mr += sg * (wr * co - wi * s);
                mi += sg * (wr * s + wi * co);
            }
    }
    // real form: rows (q, 0) = [Mr, -Mi], (q, 1) = [Mi, Mr] over columns (a, 0), (a, 1)
    const int tile = q >> 3, pq = q & 7, b = an >> 4, ai = an & 15;
    const double val[2][2] = {{mr, -mi}, {mi, mr}};
    _Float16* m16 = reinterpret_cast<_Float16*>(m);
    for (int ro = 0; ro < 2; ++ro)
        for (int ri = 0; ri < 2; ++ri) {
            const int row = 2 * pq + ro, k = 2 * ai + ri;
            const int ln = 16 * (k >> 3) + row;
            const size_t base = ((((size_t)c * (NN / 8) + tile) * nblk + b) * 2) * 64;
            const _Float16 hi = (_Float16)val[ro][ri];
            m16[(base + ln) * 8 + (k & 7)] = hi;
            m16[(base + 64 + ln) * 8 + (k & 7)] = (_Float16)(val[ro][ri] - (double)(float)hi);
        }
}

using DirFn = void (*)(DirArgs);

template <int P>
DirFn dir_pick(int nblk) {
    switch (nblk) {
        case 1: return direct_kernel<P, 1>;
        case 2: return direct_kernel<P, 2>;
        case 3: return direct_kernel<P, 3>;
        case 4: return direct_kernel<P, 4>;
    }
    return nullptr;
}

DirFn dir_select(int P, int nblk) { return P == 2 ? dir_pick<2>(nblk) : dir_pick<1>(nblk); }

int dir_groups(const SubDev& d) {
    const int ntile = d.N * d.N / 8;
    return (ntile + kDirWaves * kDirTilesPerWave - 1) / (kDirWaves * kDirTilesPerWave);
}

}  // namespace

// Launch shape of the direct form: (channel, pixel group, time chunk)
// workgroups of 4 waves, 16 pixels per wave; the chunks (one partial
// accumulator slot each) bring the launch to at least ~8 workgroups per CU.
// Arrays of at most 64 antennas on grids up to 64 whose X and Y weights are
// equal (the fragments of M for 64 antennas fill 64 registers).
hipError_t direct_configure(SubDev& d, int num_cu, int64_t max_time) {
    if (d.A > 16 * kDirMaxBlk || d.N > 64 || (d.N * d.N) % 64 != 0) return hipErrorNotSupported;
    if (!(d.P == 1 || d.wmode == kWShared)) return hipErrorNotSupported;
    d.threads = 64 * kDirWaves;
    d.lds_bytes = (size_t)2 * ((d.A + 15) / 16) * 64 * 16;
    d.prog_lds = 0;
    d.KS = 1;
    d.KK = 0;   // no transform matrix
    const int64_t base = (int64_t)d.C * dir_groups(d);
    int64_t chunks = (8LL * num_cu + base - 1) / base;
    chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, max_time));
    d.dir_chunks = (int)chunks;
    d.grid_wg = (int)(base * chunks);
    return hipSuccess;
}

int64_t direct_matrix_halfs(const SubDev& d) {
    return (int64_t)d.C * (d.N * d.N / 8) * ((d.A + 15) / 16) * 2 * 64 * 8;
}

hipError_t launch_direct_matrix(const SubDev& d, hipStream_t st) {
    const int nblk = (d.A + 15) / 16;
    const int64_t n = (int64_t)d.C * d.N * d.N * nblk * 16;
    const int bs = 256;
    direct_matrix_kernel<<<dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st>>>(
        d.cells, d.taps, d.gains, reinterpret_cast<half8*>(d.dir_m), d.C, d.A, d.P, d.K, d.N, nblk);
    return hipGetLastError();
}

hipError_t launch_direct(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st) {
    DirArgs a{};
    a.samples = samples;
    a.m = reinterpret_cast<const half8*>(d.dir_m);
    a.slots = d.slots;
    a.T = n_time;
    a.C = d.C; a.A = d.A; a.N = d.N;
    a.nblk = (d.A + 15) / 16;
    a.ntile = d.N * d.N / 8;
    a.groups = dir_groups(d);
    a.chunks = (int)std::min<int64_t>(d.dir_chunks, n_time);
    a.nibble_order = d.nibble_order;
    a.fresh = d.fresh;
    a.off_E = 0;
    DirFn fn = dir_select(d.P, a.nblk);
    if (!fn) return hipErrorNotSupported;
    const int64_t nwg = (int64_t)d.C * a.groups * a.chunks;
    hipLaunchKernelGGL(fn, dim3((unsigned)nwg), dim3(64 * kDirWaves), d.lds_bytes, st, a);
    return hipGetLastError();
}

}  // namespace epic
