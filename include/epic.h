/*
 * epic.h -- C ABI of the MI355X EPIC/MOFF imaging hot path.
 *
 * The library turns a channelised stream of 4+4-bit complex antenna voltages
 * into accumulated polarisation image cubes, following the MOFF/EPIC imaging
 * chain of Krishnan et al. (MNRAS 2023), Sec. 2 (Eq. 4) and Sec. 3:
 *
 *   unpack each 4+4-bit sample                         (Sec. 2.1)
 *   -> grid every antenna through its gridding kernel  (Eq. 4, Sec. 3.1)
 *   -> spatial 2D inverse Fourier transform            (Eq. 4, Sec. 2.2)
 *   -> square / cross-multiply the polarisations       (Eq. 5, Sec. 3.2)
 *   -> accumulate over the integration                 (Eq. 4 time average, Sec. 2.2)
 *
 * Conventions shared by every entry point:
 *   - All functions return an epic_status and never abort, throw or exit.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the plan's device (e.g. torch tensors' data_ptr()).
 *   - A hip_stream argument is a hipStream_t passed as void*; NULL means the
 *     null stream of the plan's device.  Only epic_plan and epic_destroy
 *     synchronise; every other call only enqueues work on the given stream.
 *   - A plan is not thread-safe: use one plan from one host thread at a time.
 *   - Validation happens before any side effect: a call that returns
 *     EPIC_E_ARG / EPIC_E_GEOMETRY / EPIC_E_STATE has changed nothing.
 *   - A device fault reported by the HIP runtime is returned as EPIC_E_DEVICE
 *     and is sticky: the plan refuses further work until destroyed.
 */
#ifndef EPIC_H
#define EPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EPIC_ABI_VERSION 1

typedef struct epic_plan_s* epic_plan_t;   /* opaque, owned by the library */

typedef enum {
    EPIC_OK = 0,
    EPIC_E_ARG = 1,          /* bad pointer, size, enum or combination */
    EPIC_E_GEOMETRY = 2,     /* an antenna footprint falls outside the grid */
    EPIC_E_NOMEM = 3,        /* device or host allocation failed / size overflow */
    EPIC_E_DEVICE = 4,       /* HIP runtime or kernel error (sticky) */
    EPIC_E_UNSUPPORTED = 5,  /* valid request this build does not implement */
    EPIC_E_STATE = 6         /* call not allowed in the plan's current state */
} epic_status;

/* Arithmetic of the grid / transform stages.  Accumulation is always FP32. */
typedef enum {
    EPIC_FP32 = 0,   /* FP32 vector ALU: gather gridding + register FFT */
    EPIC_FP16 = 1,   /* FP16 matrix cores (MFMA) for the transform stages; gridding as
                        the FP32 gather or as an FP16 product (hi + lo weights) */
    EPIC_FP8 = 2     /* gridding as an FP8 e4m3 product on the matrix cores (4-bit
                        samples exact in e4m3, weights as a scaled e4m3 hi + lo pair),
                        FP16 transforms; needs a GEMM gridder (AUTO selects BLOCK_GEMM) */
} epic_precision;

/* How the gridding step (Eq. 4, W_a * E_a summed over antennas) runs. */
typedef enum {
    EPIC_GRID_AUTO = 0,        /* library choice: the gather (FP32, FP16), BLOCK_GEMM (FP8) */
    EPIC_GRID_GATHER = 1,      /* each aperture cell sums its antenna list (FP32 ALU) */
    EPIC_GRID_DENSE_GEMM = 2,  /* kernel matrix [window cells x antennas] times the fields
                                  [antennas x (spectrum, pol, re/im)] on the matrix cores,
                                  every (16-cell tile, 32-antenna block) multiplied */
    EPIC_GRID_BLOCK_GEMM = 3,  /* the same product over the non-zero blocks only.  Both GEMM
                                  forms: FP16 / FP8 plans, real weights equal for both pols
                                  (else EPIC_E_UNSUPPORTED), one launch per sub-array */
    EPIC_GRID_DIRECT_GEMM = 4  /* no aperture grid and no FFT: gridding and the transform
                                  folded into one matrix per channel, each pixel's field the
                                  product of the antennas' kernel images with their fields
                                  (O(A N^2) per spectrum against O(N^2 log N), Sec. 1), FP16
                                  hi + lo on the matrix cores.  FP16 plans, at most 64
                                  antennas, grids up to 64, X and Y weights equal (else
                                  EPIC_E_UNSUPPORTED); one launch per sub-array */
} epic_gridder;

/* Output products per pixel. */
typedef enum {
    EPIC_OUT_POL = 0,     /* dual pol: XX*, YY*, Re XY*, Im XY*; single pol: XX* */
    EPIC_OUT_STOKES = 1   /* dual pol only: I, Q, U, V (linear feeds) */
} epic_output;

enum {
    EPIC_F_GRAPH = 1u,            /* replay accumulate steps from captured hipGraphs, one per
                                     (n_time, input pointers, first call after a reset or
                                     not); the 8 most recent are kept */
    EPIC_F_AUTOTUNE = 2u,         /* time candidate launch shapes at plan time: per FP16 sub-array
                                     with EPIC_GRID_AUTO the gather form (gather program in LDS
                                     or streamed from L2) against the block-GEMM form at every
                                     step size that fits; for several FP16 sub-arrays, the cost
                                     weights of the single launch and that launch against one
                                     launch per sub-array.  If the environment variable
                                     EPIC_TUNE_CACHE names a file, the choices are stored there
                                     (a JSON object keyed by device architecture and plan shape)
                                     and later plans of the same key reuse them untimed */
    EPIC_F_DRY_RUN = 4u,          /* validate and size on the CPU; touch no device */
    EPIC_F_REMOVE_AUTOCORR = 8u,  /* subtract each antenna's own power term (a = b) at read-out.
                                     Its zero-lag sums are exact int32 integers; an accumulate
                                     call that would take them past 2^24 - 1 spectra first
                                     folds them into the FP32 lag sums (also done by every
                                     read-out and epic_set_gains) */
    EPIC_F_COMPLEX_WEIGHTS = 16u, /* gather with complex weights even if every tap is real, so that
                                     epic_set_gains may pass complex (phase) gains later */
    EPIC_F_ONE_LAUNCH = 32u       /* several FP16 sub-arrays: always one persistent launch for all of
                                     them (EPIC_E_UNSUPPORTED if their shapes cannot share it).
                                     Without it they run as one launch per sub-array, unless
                                     EPIC_F_AUTOTUNE times both forms and the single launch wins */
};

/*
 * One antenna array (or band) to image.  Sec. 2.1 describes the station this
 * is shaped after: dual-polarised dipoles, 25 kHz channels, 4+4-bit samples.
 *
 * Geometry (Sec. 3.1: antennas are mapped to their nearest grid cell): for
 * channel c the centre frequency is f_c = freq0_hz + c * dfreq_hz; antenna a
 * at (x, y) metres has fractional cell coordinate
 *     g = (x * f_c / 299792458) / grid_dl + grid_n / 2      (same for y),
 * evaluated in FP64 in exactly this order without fused multiply-add, and its
 * nearest cell is floor(g + 0.5).  Its kernel covers the kernel_k x kernel_k
 * cells centred there; all of them must lie in [0, grid_n - 1] at every
 * channel, else epic_plan returns EPIC_E_GEOMETRY.  Image pixel (i, j) looks
 * at direction cosines l = (i - N/2) / (N grid_dl), m = (j - N/2) / (N grid_dl).
 */
typedef struct {
    int32_t n_ant;               /* A >= 1, A * n_pol <= 65536 */
    int32_t n_pol;               /* P: 1 or 2 (X, Y) */
    int32_t n_chan;              /* C >= 1 */
    int32_t grid_n;              /* N: multiple of 16 in [16, 256].  Kernels exist
                                    for FP32 at 16..128 (every multiple of 16),
                                    192 and 256; for FP16 with gather gridding
                                    at 32, 48, 64, 96, 128, 192 and 256; for
                                    the GEMM gridders at 32..128 of those.
                                    Other sizes: EPIC_E_UNSUPPORTED */
    int32_t kernel_k;            /* K: odd, 1..7 */
    int32_t nibble_order;        /* 0: real part in the high nibble; 1: swapped */
    double grid_dl;              /* grid spacing in wavelengths (> 0) */
    double freq0_hz;             /* centre frequency of channel 0 (> 0) */
    double dfreq_hz;             /* channel spacing (>= 0) */
    const double* ant_xy_m;      /* host [A][2] east, north in metres; copied */
    const float* taps;           /* host [C][A][P][K][K][2] complex kernel taps
                                    (row-major [dy][dx], re/im), or NULL for the
                                    default Gaussian; copied */
    double kernel_sigma_cells;   /* Gaussian sigma in cells when taps == NULL
                                    (<= 0 selects 0.5).  The Gaussian weighs tap
                                    (dx, dy) by exp(-d^2 / (2 sigma^2)), d the
                                    distance from the tap's cell centre to g,
                                    normalised to unit sum. */
} epic_array_desc;

typedef struct {
    int32_t n_sub;                 /* number of arrays / bands, 1..16 */
    const epic_array_desc* sub;    /* host [n_sub]; copied */
    int32_t precision;             /* epic_precision */
    int32_t gridder;               /* epic_gridder */
    int32_t output;                /* epic_output */
    int32_t device;                /* HIP device ordinal */
    int64_t max_time;              /* largest n_time a single accumulate call may pass (>= 1) */
    uint32_t flags;                /* EPIC_F_* */
    int32_t reserved[4];           /* must be zero */
} epic_plan_desc;

/* Plan facts for callers and tests (all sizes in bytes). */
typedef struct {
    int32_t n_sub;
    int32_t precision, gridder, output;
    int32_t npp[16];               /* products per pixel per sub-array (1 or 4) */
    int32_t slots[16];             /* time slots (partial accumulators) per sub-array */
    int32_t window_max[16];        /* largest aperture window side over channels */
    int32_t threads[16];           /* workgroup size of the sub-array's kernel */
    int64_t device_bytes;          /* device memory owned by the plan */
    int64_t lds_bytes[16];         /* LDS per workgroup of each sub-array's kernel */
    int32_t graph;                 /* 1 if accumulate replays a hipGraph */
    int32_t autotuned;             /* 1: launch forms / work split timed at plan time;
                                      2: taken from the EPIC_TUNE_CACHE file */
    int32_t batched;               /* 1 if all sub-arrays run in one launch */
    int32_t weight[16];            /* batched: cost of one spectrum per sub-array */
    int32_t col_split[16];         /* KS: workgroups sharing one spectrum's image columns */
    int32_t workgroups[16];        /* persistent workgroups of the sub-array's launch */
    int32_t can_batch;             /* 1 if the one-launch form exists for these sub-arrays */
    double form_ms[2];             /* autotuner: probe call time, one launch / one per sub-array */
    int32_t grid_form[16];         /* epic_gridder each sub-array's kernel runs */
    int32_t grid_step[16];         /* spectra per gridding product (1 for the gather, 16 / n_pol
                                      for the direct form) */
    int32_t graph_builds;          /* EPIC_F_GRAPH: graphs captured so far */
    int32_t autocorr_pending[16];  /* EPIC_F_REMOVE_AUTOCORR: spectra in the zero-lag sums
                                      since their last fold */
    int32_t autocorr_fold_limit;   /* the count at which they are folded before a call */
    int64_t grid_blocks[16];       /* GEMM gridding: (tile, antenna block) products per spectrum
                                      step and column part, summed over channels */
} epic_plan_info;

/*
 * epic_plan -- validate the arrays, compute the geometry (Sec. 3.1 nearest-cell
 * mapping) in FP64 on the host, compute the kernel taps and transform tables
 * in FP64 on the device, and allocate the accumulators.
 *   desc        host, read during the call only.
 *   hip_stream  stream for the one-off device set-up (synchronised before return).
 *   out         host; receives the new plan on EPIC_OK, NULL otherwise.
 * Errors: EPIC_E_ARG (bad field, non-zero reserved), EPIC_E_GEOMETRY,
 * EPIC_E_NOMEM, EPIC_E_DEVICE, EPIC_E_UNSUPPORTED (e.g. a grid size with no
 * kernel).  With EPIC_F_DRY_RUN no HIP call is made; the plan can be queried
 * and destroyed but accumulate / readout return EPIC_E_STATE.
 * The accumulators start at zero.
 */
epic_status epic_plan(const epic_plan_desc* desc, void* hip_stream, epic_plan_t* out);

/*
 * epic_grid_fft_accumulate -- the hot path.  For every sub-array, channel and
 * time sample: unpack, grid (Eq. 4), 2D transform (Eq. 4), form the
 * polarisation products (Eq. 5) and add them into the plan's FP32 accumulators
 * (the time sum of Eq. 4; no 1/T normalisation).
 *   d_samples   host array [n_sub] of device pointers; sub-array s points at
 *               uint8 [n_time][C_s][A_s][P_s] bytes, one 4+4-bit complex
 *               sample each (two's complement nibbles).  Read only; must stay
 *               valid until the stream passes this call.
 *   n_time      0..max_time spectra (0 is a no-op).
 * Errors: EPIC_E_ARG (NULL pointer, n_time out of range), EPIC_E_STATE (dry
 * run or sticky error), EPIC_E_DEVICE (launch failure).
 */
epic_status epic_grid_fft_accumulate(epic_plan_t plan, const uint8_t* const* d_samples,
                                     int64_t n_time, void* hip_stream);

/*
 * epic_readout -- reduce the plan's partial accumulators in a fixed order into
 * the caller's image cubes, then optionally zero them (start a new integration).
 *   d_images    host array [n_sub] of device pointers; sub-array s receives
 *               float [C_s][NPP_s][N_s][N_s], indexed [c][product][j][i]
 *               (j: m axis, i: l axis).  Products: EPIC_OUT_POL dual pol
 *               XX*, YY*, Re XY*, Im XY*; single pol XX*; EPIC_OUT_STOKES
 *               I = XX*+YY*, Q = XX*-YY*, U = 2 Re XY*, V = 2 Im XY*
 *               (linear feeds, XY* = (U + iV)/2: a field with E_Y = -i E_X
 *               has V = +I, one with E_Y = +i E_X has V = -I).
 *               Overwritten; must stay valid until the stream passes the call.
 *   reset       non-zero: zero the accumulators after reading.
 * Errors: EPIC_E_ARG, EPIC_E_STATE, EPIC_E_DEVICE.
 */
epic_status epic_readout(epic_plan_t plan, float* const* d_images, int32_t reset, void* hip_stream);

/*
 * epic_efield -- electric-field images instead of accumulated products (the
 * method can emit field images as well as intensity images, Sec. 1): for every
 * spectrum t, channel c and polarisation p of sub-array `sub`, the transform
 * FT^-1[sum_a W_a * E_a] of Eq. 4 before squaring, with the (-1)^(x+y) grid
 * centring, i.e. the field whose squared magnitude summed over t is the XX*
 * (or YY*) image of epic_readout.
 *   d_samples   device uint8 [n_time][C][A][P] of this sub-array.
 *   d_out       device float [n_time][C][P][N][N][2] (re, im), indexed
 *               [t][c][p][j][i] with pixels as for epic_readout; overwritten.
 *   n_time      0..max_time (0 is a no-op).
 * Enqueued on hip_stream; the plan's accumulators are untouched.  FP32 plans
 * only (EPIC_E_UNSUPPORTED otherwise).
 * Errors: EPIC_E_ARG, EPIC_E_STATE, EPIC_E_UNSUPPORTED, EPIC_E_DEVICE.
 */
epic_status epic_efield(epic_plan_t plan, int32_t sub, const uint8_t* d_samples, int64_t n_time, float* d_out,
                        void* hip_stream);

/*
 * epic_set_gains -- per-antenna complex gains (delay / phase / amplitude
 * corrections, Sec. 2.2's delay correction step) folded into the kernel taps
 * of one sub-array: tap'(c, a, p) = g(c, a, p) * tap(c, a, p).  Replaces any
 * previous gains (NULL restores unit gains).  Enqueued on hip_stream; later
 * accumulate calls on the same stream see the new taps.
 *   h_gains     host float [C][A][P][2] (re, im); copied before return.
 * Errors: EPIC_E_ARG, EPIC_E_STATE, EPIC_E_DEVICE.
 */
epic_status epic_set_gains(epic_plan_t plan, int32_t sub, const float* h_gains, void* hip_stream);

/*
 * epic_image_noalloc -- one whole integration that allocates no device memory,
 * for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It computes what
 * epic_grid_fft_accumulate(plan, d_samples, n_time) on zeroed accumulators
 * followed by epic_readout(plan, d_images, reset) gives, but keeps the partial
 * accumulators in a static device buffer of the library (at most
 * EPIC_NOALLOC_MAX_BYTES per GPU, held from the library's first plan on that
 * GPU until the process ends) instead of the plan's, which it leaves
 * untouched.  Several sub-arrays run as one launch each (also in plans that
 * would batch them).
 *   d_samples   host array [n_sub] of device pointers, as for accumulate.
 *   n_time      0..max_time (0 writes all-zero images).
 *   d_images    host array [n_sub] of device pointers, as for epic_readout;
 *               overwritten.
 * The buffer is cleared at the start of every call.  Every call on one GPU
 * shares that GPU's buffer: calls that overlap in time on one GPU (other
 * streams, other plans, other host threads) race and give wrong images.
 * Errors: EPIC_E_ARG, EPIC_E_STATE, EPIC_E_DEVICE; EPIC_E_NOMEM when the
 * plan's partial accumulators for n_time spectra, sum over sub-arrays of
 * S x C x NPP x N x N floats, exceed EPIC_NOALLOC_MAX_BYTES; EPIC_E_UNSUPPORTED
 * for plans with EPIC_F_REMOVE_AUTOCORR (whose zero-lag sums are plan state).
 */
#define EPIC_NOALLOC_MAX_BYTES (64ll << 20)
epic_status epic_image_noalloc(epic_plan_t plan, const uint8_t* const* d_samples, int64_t n_time,
                               float* const* d_images, void* hip_stream);

/* epic_plan_query -- fill *info (host).  Works on dry-run plans.  EPIC_E_ARG on NULL. */
epic_status epic_plan_query(epic_plan_t plan, epic_plan_info* info);

/*
 * epic_debug_geometry -- copy the plan's nearest-cell indices of sub-array
 * `sub` to host int32 [C][A][2] (x, y) for bit-exact comparison.  Works on
 * dry-run plans.  EPIC_E_ARG on bad arguments.
 */
epic_status epic_debug_geometry(epic_plan_t plan, int32_t sub, int32_t* h_cells);

/*
 * epic_debug_schedule -- the work split of one accumulate call of n_time
 * spectra, computed on the host with the same functions the kernels use.
 * For sub-array `sub` and every spectrum index k = v * n_time + t (virtual
 * channel v = c * KS + column part, KS = col_split from epic_plan_query) it
 * writes the owning workgroup to h_wg[k] and the partial-accumulator slot
 * that workgroup adds it into to h_slot[k]; both arrays hold
 * n_chan * KS * n_time int32 values.  Works on dry-run plans.  EPIC_E_ARG on
 * bad arguments or n_time outside [1, max_time]; EPIC_E_STATE if the split
 * gives a spectrum two owners or none, or a slot outside [0, slots).
 */
epic_status epic_debug_schedule(epic_plan_t plan, int32_t sub, int64_t n_time, int32_t* h_wg, int32_t* h_slot);

/*
 * epic_debug_unpack -- run the device 4+4-bit decoder of the hot path on n
 * bytes: d_out (device float [n][2]) receives (re, im).  Enqueued on
 * hip_stream.  EPIC_E_ARG on NULL pointers or n < 0; EPIC_E_DEVICE on launch
 * failure.
 */
epic_status epic_debug_unpack(const uint8_t* d_bytes, int64_t n, int32_t nibble_order,
                              float* d_out, void* hip_stream);

/* epic_destroy -- synchronise the plan's device, free everything.  NULL is a no-op. */
epic_status epic_destroy(epic_plan_t plan);

/* epic_status_str -- static, NUL-terminated name of a status code. */
const char* epic_status_str(epic_status status);

/* epic_abi_version -- EPIC_ABI_VERSION of the built library. */
int32_t epic_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EPIC_H */
