// Internal declarations shared by the host plan (plan.cpp) and the HIP kernel
// translation units.  Not part of the public ABI (include/epic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/epic.h"

namespace epic {

constexpr int kMaxSub = 16;
constexpr int kMaxGridN = 256;

// Aperture window of one (sub-array, channel): the bounding box of every
// antenna's kernel footprint.  Cells outside it are identically zero, so the
// transform only reads the window.  Because a cyclic shift of the aperture
// multiplies both polarisations' sky fields by the same unit phase, the
// products of Eq. 5 do not depend on where the window sits in the grid; the
// kernels place it at the origin.
//
// Gridding runs as a "gather program": the non-empty window cells, sorted by
// their number of contributions (so neighbouring lanes loop equally long),
// each with a list of (antenna, tap) contributions padded with zero-weight
// entries to whole groups of kGroup.
constexpr int kGroup = 4;

struct ChanInfo {
    int32_t x0, y0;      // absolute cell of window element (0, 0)
    int32_t R, W;        // window rows (y extent) and columns (x extent)
    int32_t n_cell;      // non-empty cells
    int32_t cell_off;    // offset of this channel's cell descriptors
    int32_t n_grp;       // groups of kGroup entries
    int32_t grp_off;     // offset of this channel's first group
};

// Cell descriptor: x = LDS float2 offset of the cell within one pol's window
// (row * pitch + col) | (groups << 16); y = first group (channel-relative).
using CellDesc = uint2;

// Operand types of the GEMM-gridding form (gridding on the matrix cores).
constexpr int kBgFp16 = 0, kBgFp8 = 1;

// GEMM-gridding tables of one channel: its cell tiles (16 non-empty window
// cells each, in raster order) and the (tile, antenna block) pairs it
// multiplies -- the non-zero ones (block-sparse form) or all of them (dense).
struct BgChan {
    int32_t tile_off;    // first tile of this channel in the tile and cell tables
    int32_t n_tile;
    int32_t ent_off;     // first block entry of this channel
    int32_t n_ent;
};

// Device resources of one sub-array.
struct SubDev {
    // shape
    int A, P, C, N, K, NPP, nibble_order;
    int S;               // partial accumulator slots per channel
    int KS;              // column split of the image across workgroups
    int Rmax, Wmax;      // largest window over channels
    int WP;              // LDS row pitch (float2) of the gridded window
    int Gmax, CellMax;   // largest group / non-empty cell count over channels
    int wmode;           // gather weights: 0 complex, 1 real per pol, 2 real shared by both pols
    int grid_wg;         // resident workgroups of one launch (persistent)
    // tables
    ChanInfo* chans;          // [C]
    CellDesc* cells_desc;     // [sum n_cell]
    uint16_t* grp_ant;        // [sum n_grp * kGroup] antenna per entry (0 for padding)
    uint8_t* grp_tap;         // [sum n_grp * kGroup] tap dy*K+dx, 255 for padding
    float* grp_w;             // [sum n_grp * kGroup][WF] entry weights, WF = 2P, P or 1 by wmode
    int32_t* cells;           // [C][A][2] nearest cell
    double* gfrac;            // [C][A][2] fractional cell coordinate
    float* taps;              // [C][A][P][K][K][2] FP32 taps (before gains)
    float* gains;             // [C][A][P][2] complex gains in effect (or nullptr = unit)
    float* gains_buf = nullptr;   // device storage of the gains once any were set
    float2* twiddle;          // [N] exp(+2 pi i r / N)
    float* slots;             // [S][C][NPP][N][N] partial accumulators
    int32_t* vaa = nullptr;   // [C][A][4 or 1] zero-lag antenna correlations (autocorrelation removal)
    float* lag = nullptr;     // [C][(2K-1)^2][3 or 1][2] lag sums of the autocorrelation image
    // launch shape
    int threads;
    size_t lds_bytes;
    int prog_lds;        // gather program copied to LDS (else read through L2)
    int smp_bufs = 2;    // FP32: decoded sample buffers (2: decode overlaps gridding)
    // matrix-core (reduced precision) form
    int precision;       // epic_precision of this sub-array's kernel
    int KK;              // 32-deep MFMA steps per transform product
    void* dft16;         // [2N][32 KK] FP16 real-form DFT matrix
    // gridding on the matrix cores (EPIC_GRID_DENSE_GEMM / EPIC_GRID_BLOCK_GEMM)
    int gridder = EPIC_GRID_GATHER;   // gridding form this sub-array's kernel runs
    int R4max = 0;                    // largest window row count, rounded up to 4
    int bg_tb = 1;                    // spectra per gridding step
    int bg_nablk = 0;                 // antenna blocks of 32
    int64_t bg_nentries = 0;          // gather entries (length of bg_dst)
    int64_t bg_nent = 0;              // block entries over all channels
    BgChan* bg_chans = nullptr;       // [C]
    uint2* bg_tiles = nullptr;        // [tiles] (first block entry, channel-relative; block count)
    uint16_t* bg_cells = nullptr;     // [tiles][16] (r << 8 | w), 0xFFFF padding
    uint16_t* bg_ents = nullptr;      // [entries] antenna block of each block entry
    int32_t* bg_perm = nullptr;       // [A] antenna at raster position s
    int32_t* bg_dst = nullptr;        // [gather entries] operand element of each entry, -1 padding
    unsigned char* bg_w = nullptr;    // [terms][entries][64 lanes][8] split weights, high part first
    int bg_nterm = 2;                 // terms of the split (FP16: 2, FP8: 3)
    float* bg_scale = nullptr;        // [2] FP8 weight scale and its inverse
    // direct imaging (EPIC_GRID_DIRECT_GEMM): per-channel kernel-image matrix
    void* dir_m = nullptr;            // [C][N^2 / 8][A / 16][2 terms][64 lanes][8] FP16
    int dir_chunks = 1;               // time chunks (partial accumulator slots) of a launch
    int fresh = 0;                    // per call: the slots hold zeros (stores replace adds)
};

// One sub-array as seen by the batched (several sub-arrays in one launch)
// matrix-core kernel; a device copy of the table is passed to the kernel.
struct BatchSub {
    const ChanInfo* chans;
    const CellDesc* cells_desc;
    const uint16_t* grp_ant;
    const float* grp_w;
    const uint16_t* dft;      // FP16 real-form DFT matrix [2N][32 KK]
    float* slots;             // [S][C][NPP][N][N]
    int C, A, V;              // channels, antennas, virtual channels (C * KS)
    int N, KK, KS, NK, IT, WAVES, NT1, WP, M1max;
    int nibble_order, S, weight, prog_lds;
};

// Launch state of a batched plan.
struct BatchDev {
    BatchSub* table;          // device [n_sub]
    int grid_wg, threads, kkmax, P, wmode, prog_lds, smp_stride;
    size_t lds_bytes;
    uint32_t off[6];
    int fresh = 0;            // per call: the slots hold zeros (stores replace adds)
};

// ---- launchers (defined in the .hip translation units) -----------------

// One-off FP64 set-up on the device.
hipError_t launch_gaussian_taps(const SubDev& d, double sigma, hipStream_t st);
hipError_t launch_twiddles(const SubDev& d, hipStream_t st);
hipError_t launch_entry_weights(const SubDev& d, hipStream_t st);

// The FP32 hot path for one sub-array: n_time spectra of uint8 [T][C][A][P].
// fp32_configure picks the launch shape; with device < 0 it makes no HIP call.
hipError_t fp32_configure(SubDev& d, int device, int num_cu);
hipError_t launch_fp32(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st,
                       float* efield = nullptr);

// The FP16 matrix-core hot path (same contract as launch_fp32).
// force_prog: -1 library choice, 0 / 1 gather program streamed from L2 / in LDS
hipError_t mfma_configure(SubDev& d, int device, int num_cu, int force_prog = -1);
hipError_t launch_dft_matrix(const SubDev& d, hipStream_t st);
hipError_t launch_mfma(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st);

// Gridding on the matrix cores (kernels_bgemm.hip): launch shape, the split
// operand weights (after launch_entry_weights), and the hot path.
// force_tb: 0 library choice, else that many spectra per gridding step
hipError_t bg_configure(SubDev& d, int device, int num_cu, int force_tb = 0);
hipError_t launch_bg_weights(const SubDev& d, hipStream_t st);
hipError_t launch_bgemm(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st);

// Direct imaging on the matrix cores (kernels_direct.hip): launch shape,
// the kernel-image matrix (FP64, split FP16 hi + lo), and the hot path.
hipError_t direct_configure(SubDev& d, int num_cu, int64_t max_time);
int64_t direct_matrix_halfs(const SubDev& d);
hipError_t launch_direct_matrix(const SubDev& d, hipStream_t st);
hipError_t launch_direct(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st);

// Several FP16 sub-arrays in one persistent launch.
hipError_t batch_configure(SubDev* subs, int n_sub, BatchDev& bd, int device, int num_cu);
BatchSub batch_entry(const SubDev& d, int weight);
hipError_t launch_batch(const BatchDev& bd, const uint8_t* const* samples, int n_sub, int64_t n_time,
                        hipStream_t st);

// Ordered reduction of the slots into [C][NPP][N][N] (or Stokes), optional reset.
hipError_t launch_autocorr(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st);
hipError_t launch_autocorr_fold(const SubDev& d, hipStream_t st);
hipError_t launch_zero(float* x, int64_t n, hipStream_t st);
int64_t vaa_count(const SubDev& d);
int64_t lag_count(const SubDev& d);
hipError_t launch_readout(const SubDev& d, float* out, int stokes, int reset, hipStream_t st);

// Debug decode of n bytes into float (re, im) pairs.
hipError_t launch_unpack_debug(const uint8_t* in, int64_t n, int order, float* out, hipStream_t st);

}  // namespace epic
