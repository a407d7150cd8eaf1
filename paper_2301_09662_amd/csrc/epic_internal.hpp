// Internal declarations shared by the host plan (plan.cpp) and the HIP kernel
// translation units.  Not part of the public ABI (include/epic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/epic.h"

namespace epic {

constexpr int kMaxSub = 16;
constexpr int kMaxGridN = 128;

// Aperture window of one (sub-array, channel): the bounding box of every
// antenna's kernel footprint.  Cells outside it are identically zero, so the
// transform only reads the window.  Because a cyclic shift of the aperture
// multiplies both polarisations' sky fields by the same unit phase, the
// products of Eq. 5 do not depend on where the window sits in the grid; the
// kernels place it at the origin.
struct ChanInfo {
    int32_t x0, y0;      // absolute cell of window element (0, 0)
    int32_t R, W;        // window rows (y extent) and columns (x extent)
    int32_t cell_off;    // offset of this channel's cell_ptr block (R*W + 1 words)
    int32_t ent_off;     // offset of this channel's first gather entry
    int32_t n_ent;       // entries of this channel (A * K * K)
    int32_t pad;
};

// Device resources of one sub-array.
struct SubDev {
    // shape
    int A, P, C, N, K, NPP, nibble_order;
    int S;               // time slots (partial accumulators)
    int KS;              // column split of the image across workgroups
    int Rmax, Wmax, Emax;  // largest window / entry count over channels
    // tables
    ChanInfo* chans;          // [C]
    uint32_t* cell_ptr;       // per channel [R*W + 1], entry offsets relative to ent_off
    uint16_t* ent_ant;        // [sum n_ent] antenna of each gather entry
    uint8_t* ent_tap;         // [sum n_ent] tap index dy*K + dx
    float* ent_w;             // [sum n_ent][2P] weight of each entry per pol (re, im)
    int32_t* cells;           // [C][A][2] nearest cell
    double* gfrac;            // [C][A][2] fractional cell coordinate
    float* taps;              // [C][A][P][K][K][2] FP32 taps (before gains)
    float* gains;             // [C][A][P][2] complex gains (or nullptr = unit)
    float2* twiddle;          // [N] exp(+2 pi i r / N)
    float* slots;             // [S][C][NPP][N][N] partial accumulators
    // launch shape
    int threads;
    size_t lds_bytes;
    int csr_in_lds;
};

// ---- launchers (defined in the .hip translation units) -----------------

// One-off FP64 set-up on the device.
hipError_t launch_gaussian_taps(const SubDev& d, double sigma, hipStream_t st);
hipError_t launch_twiddles(const SubDev& d, hipStream_t st);
hipError_t launch_entry_weights(const SubDev& d, hipStream_t st);

// The FP32 hot path for one sub-array: n_time spectra of uint8 [T][C][A][P].
hipError_t fp32_configure(SubDev& d, int device);
hipError_t launch_fp32(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st);

// Ordered reduction of the slots into [C][NPP][N][N] (or Stokes), optional reset.
hipError_t launch_readout(const SubDev& d, float* out, int stokes, int reset, hipStream_t st);

// Debug decode of n bytes into float (re, im) pairs.
hipError_t launch_unpack_debug(const uint8_t* in, int64_t n, int order, float* out, hipStream_t st);

}  // namespace epic
