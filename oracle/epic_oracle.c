/*
 * epic_oracle.c -- plain FP64 CPU reference of the EPIC/MOFF image.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the GPU path.
 *
 * What it computes (paper Sec. 2, Eq. 4, with the polarisation products of
 * Sec. 3.2 / Eq. 5), per channel c and time sample t:
 *
 *   1. unpack each 4+4-bit sample into a complex integer (Sec. 2.1);
 *   2. grid every antenna's field onto a regular aperture grid through its
 *      gridding kernel W_a (the convolution W_a * E_a of Eq. 3/4, summed over
 *      antennas), each cell also multiplied by (-1)^(x+y) so that the image
 *      centre lands on pixel N/2;
 *   3. take the spatial 2D transform FT^-1 of Eq. 4 as a textbook DFT,
 *      exp(+2 pi i (x i + y j) / N), unnormalised, rows then columns;
 *   4. square / cross-multiply the two polarisation images pixel by pixel
 *      (XX*, YY*, and the real and imaginary parts of XY*) and sum over t,
 *      which is the time average of Eq. 4 without the 1/T.
 *
 * Readings of the paper that this file fixes (the paper leaves them open):
 *   - the nearest grid cell of an antenna is floor(g + 0.5) of its fractional
 *     cell coordinate g = (x f_c / c0) / dl + N/2 (Sec. 3.1 maps antennas to
 *     their nearest grid cell), evaluated in this exact operation order with
 *     no fused multiply-add;
 *   - the default kernel is a K x K Gaussian of the distance between each tap
 *     centre and the antenna, sigma in cells, normalised to unit sum;
 *   - a nibble pair is two's complement, real part in the high nibble unless
 *     nibble_order == 1;
 *   - the fourth product printed in Sec. 3.2 is the conjugate of XY*, so the
 *     stored products are XX*, YY*, Re XY*, Im XY* (single pol: XX* only);
 *   - a footprint cell outside [0, N-1] is an error (no wrap, no clip).
 *
 * Pins (tests/test_oracle.py; each checks the function against something
 * other than itself, and the planted-mistake tests show that a dropped term,
 * a wrong sign, a transposed operand, a swapped conjugate or nibble, a lost
 * checkerboard or normalisation, or truncation instead of rounding, each
 * fails at least one of them):
 *   ora_unpack_table    every byte against the two's-complement table, both
 *                       nibble orders;
 *   ora_geometry        closed-form positions (centre, whole cells, ties),
 *                       scaling with frequency, out-of-grid refusal;
 *   ora_taps            the Gaussian's closed form, its shift with the
 *                       sub-cell offset, user taps passed through;
 *   ora_dft2            numpy's inverse FFT times N^2, and the orientation of
 *                       a single-cell grid's plane wave;
 *   ora_grid, ora_image_range
 *                       FX brute force (per-pair correlations imaged
 *                       directly, Eq. 3 with Eq. 4), the worked example's
 *                       closed form (tests/golden/worked_example.txt),
 *                       Parseval, Y = i X conjugation order, invariants and
 *                       linearity, point-source localisation;
 *   ora_autocorr_range  FX imaging with the a = b terms dropped, and the sum
 *                       of one-antenna images;
 *   ora_efield_range    a lone antenna's field equals its kernel image, and
 *                       the products of the fields sum to ora_image_range.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_C0 299792458.0
#define ORA_PI 3.14159265358979323846

enum { ORA_OK = 0, ORA_E_ARG = 1, ORA_E_GEOMETRY = 2, ORA_E_NOMEM = 3 };

typedef struct {
    int32_t n_ant, n_pol, n_chan, grid_n, kernel_k, nibble_order;
    double grid_dl, freq0_hz, dfreq_hz, kernel_sigma_cells;
    const double* ant_xy;   /* [A][2] east, north in metres */
    const float* taps;      /* [C][A][P][K][K][2] complex, or NULL for Gaussian */
} ora_array;

/* ---- step 1: 4+4-bit unpack ------------------------------------------- */
static int nibble_value(unsigned v) { return v >= 8u ? (int)v - 16 : (int)v; }

static void unpack(uint8_t b, int order, double* re, double* im) {
    int hi = nibble_value((b >> 4) & 0xFu);
    int lo = nibble_value(b & 0xFu);
    if (order == 0) { *re = hi; *im = lo; } else { *re = lo; *im = hi; }
}

int ora_unpack_table(int nibble_order, double* re, double* im) {
    for (int b = 0; b < 256; ++b) unpack((uint8_t)b, nibble_order, &re[b], &im[b]);
    return ORA_OK;
}

static int check_array(const ora_array* s) {
    if (!s || !s->ant_xy) return ORA_E_ARG;
    if (s->n_ant < 1 || (s->n_pol != 1 && s->n_pol != 2) || s->n_chan < 1) return ORA_E_ARG;
    if (s->grid_n < 2 || (s->grid_n & 1) || s->kernel_k < 1 || !(s->kernel_k & 1)) return ORA_E_ARG;
    if (!(s->grid_dl > 0.0) || !(s->freq0_hz > 0.0)) return ORA_E_ARG;
    return ORA_OK;
}

/* ---- step 2a: geometry (nearest cell, fractional coordinate) ---------- */
int ora_geometry(const ora_array* s, int32_t* cell /*[C][A][2]*/, double* g /*[C][A][2]*/) {
    int rc = check_array(s);
    if (rc) return rc;
    const int N = s->grid_n, h = s->kernel_k / 2;
    int bad = 0;
    for (int c = 0; c < s->n_chan; ++c) {
        double f = s->freq0_hz + (double)c * s->dfreq_hz;
        for (int a = 0; a < s->n_ant; ++a) {
            for (int ax = 0; ax < 2; ++ax) {
                double u = s->ant_xy[2 * a + ax] * f / ORA_C0;   /* wavelengths */
                double gg = u / s->grid_dl + 0.5 * (double)N;     /* cells */
                double p = floor(gg + 0.5);
                size_t o = ((size_t)c * s->n_ant + a) * 2 + ax;
                g[o] = gg;
                cell[o] = (int32_t)p;
                if (p - h < 0.0 || p + h > (double)(N - 1)) bad = 1;
            }
        }
    }
    return bad ? ORA_E_GEOMETRY : ORA_OK;
}

/* ---- step 2b: gridding kernel taps ------------------------------------ */
/* taps_out: [C][A][P][K][K][2] in FP64.  User taps are promoted from FP32. */
int ora_taps(const ora_array* s, const int32_t* cell, const double* g, double* taps_out) {
    int rc = check_array(s);
    if (rc) return rc;
    const int A = s->n_ant, P = s->n_pol, K = s->kernel_k, h = K / 2;
    const size_t per_ant = (size_t)P * K * K * 2;
    for (int c = 0; c < s->n_chan; ++c) {
        for (int a = 0; a < A; ++a) {
            double* w = taps_out + ((size_t)c * A + a) * per_ant;
            if (s->taps) {
                const float* src = s->taps + ((size_t)c * A + a) * per_ant;
                for (size_t k = 0; k < per_ant; ++k) w[k] = (double)src[k];
                continue;
            }
            size_t o = ((size_t)c * A + a) * 2;
            double sig = s->kernel_sigma_cells > 0.0 ? s->kernel_sigma_cells : 0.5;
            double sum = 0.0;
            for (int dy = -h; dy <= h; ++dy)
                for (int dx = -h; dx <= h; ++dx) {
                    double ex = (double)(cell[o + 0] + dx) - g[o + 0];
                    double ey = (double)(cell[o + 1] + dy) - g[o + 1];
                    double v = exp(-(ex * ex + ey * ey) / (2.0 * sig * sig));
                    w[((dy + h) * K + (dx + h)) * 2 + 0] = v;
                    w[((dy + h) * K + (dx + h)) * 2 + 1] = 0.0;
                    sum += v;
                }
            for (int k = 0; k < K * K; ++k) w[2 * k] /= sum;
            for (int p = 1; p < P; ++p)
                memcpy(w + (size_t)p * K * K * 2, w, sizeof(double) * K * K * 2);
        }
    }
    return ORA_OK;
}

/* ---- step 2c: grid one polarisation of one (c, t) row ----------------- */
/* row: [A][P] bytes; taps_c: [A][P][K][K][2]; cell_c: [A][2]; grid: [N][N][2] */
int ora_grid(const ora_array* s, const double* taps_c, const int32_t* cell_c,
             const uint8_t* row, int p, double* grid) {
    const int N = s->grid_n, A = s->n_ant, P = s->n_pol, K = s->kernel_k, h = K / 2;
    memset(grid, 0, sizeof(double) * 2 * N * N);
    for (int a = 0; a < A; ++a) {
        double er, ei;
        unpack(row[a * P + p], s->nibble_order, &er, &ei);
        const double* w = taps_c + ((size_t)a * P + p) * K * K * 2;
        for (int dy = -h; dy <= h; ++dy)
            for (int dx = -h; dx <= h; ++dx) {
                int x = cell_c[2 * a + 0] + dx, y = cell_c[2 * a + 1] + dy;
                double sgn = ((x + y) & 1) ? -1.0 : 1.0;
                double wr = w[((dy + h) * K + (dx + h)) * 2 + 0];
                double wi = w[((dy + h) * K + (dx + h)) * 2 + 1];
                grid[(y * N + x) * 2 + 0] += sgn * (wr * er - wi * ei);
                grid[(y * N + x) * 2 + 1] += sgn * (wr * ei + wi * er);
            }
    }
    return ORA_OK;
}

/* ---- step 3: textbook 2D DFT, exp(+2 pi i (x i + y j)/N) --------------- */
static void twiddle_table(int N, double* tw) {
    for (int r = 0; r < N; ++r) {
        tw[2 * r + 0] = cos(2.0 * ORA_PI * (double)r / (double)N);
        tw[2 * r + 1] = sin(2.0 * ORA_PI * (double)r / (double)N);
    }
}

/* in/out: [N][N][2] indexed [y][x] -> [j][i]; tmp: [N][N][2] scratch */
static void dft2(int N, const double* tw, const double* in, double* tmp, double* out) {
    /* rows: for each y, transform along x */
    for (int y = 0; y < N; ++y)
        for (int i = 0; i < N; ++i) {
            double ar = 0.0, ai = 0.0;
            for (int x = 0; x < N; ++x) {
                const double* t = tw + 2 * (((long)x * i) % N);
                double vr = in[(y * N + x) * 2], vi = in[(y * N + x) * 2 + 1];
                ar += vr * t[0] - vi * t[1];
                ai += vr * t[1] + vi * t[0];
            }
            tmp[(y * N + i) * 2] = ar;
            tmp[(y * N + i) * 2 + 1] = ai;
        }
    /* columns: for each i, transform along y */
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double ar = 0.0, ai = 0.0;
            for (int y = 0; y < N; ++y) {
                const double* t = tw + 2 * (((long)y * j) % N);
                double vr = tmp[(y * N + i) * 2], vi = tmp[(y * N + i) * 2 + 1];
                ar += vr * t[0] - vi * t[1];
                ai += vr * t[1] + vi * t[0];
            }
            out[(j * N + i) * 2] = ar;
            out[(j * N + i) * 2 + 1] = ai;
        }
}

int ora_dft2(int N, const double* in, double* out) {
    if (N < 1) return ORA_E_ARG;
    double* tw = (double*)malloc(sizeof(double) * 2 * N);
    double* tmp = (double*)malloc(sizeof(double) * 2 * N * N);
    if (!tw || !tmp) { free(tw); free(tmp); return ORA_E_NOMEM; }
    twiddle_table(N, tw);
    dft2(N, tw, in, tmp, out);
    free(tw);
    free(tmp);
    return ORA_OK;
}

/* ---- steps 1-4 for a whole call ---------------------------------------- */
/*
 * samples: uint8 [T][C][A][P]; out: FP64 [C][NPP][N][N] (overwritten), NPP = 1
 * for single pol (XX*) and 4 for dual pol (XX*, YY*, Re XY*, Im XY*).
 * chan_begin/chan_end restrict the work to a channel range (others are left
 * untouched); n_threads <= 0 lets OpenMP choose.
 */
int ora_image_range(const ora_array* s, const uint8_t* samples, int64_t T,
                    int chan_begin, int chan_end, double* out, int n_threads) {
    int rc = check_array(s);
    if (rc) return rc;
    if (!samples || !out || T < 0) return ORA_E_ARG;
    if (chan_begin < 0 || chan_end > s->n_chan || chan_begin > chan_end) return ORA_E_ARG;
    const int N = s->grid_n, A = s->n_ant, P = s->n_pol, C = s->n_chan, K = s->kernel_k;
    const int NPP = (P == 2) ? 4 : 1;
    const size_t NN = (size_t)N * N;

    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)C * A * 2);
    double* g = (double*)malloc(sizeof(double) * (size_t)C * A * 2);
    double* taps = (double*)malloc(sizeof(double) * (size_t)C * A * P * K * K * 2);
    double* tw = (double*)malloc(sizeof(double) * 2 * N);
    if (!cell || !g || !taps || !tw) { free(cell); free(g); free(taps); free(tw); return ORA_E_NOMEM; }
    rc = ora_geometry(s, cell, g);
    if (rc == ORA_OK) rc = ora_taps(s, cell, g, taps);
    if (rc != ORA_OK) { free(cell); free(g); free(taps); free(tw); return rc; }
    twiddle_table(N, tw);

    int nomem = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int c = chan_begin; c < chan_end; ++c) {
        double* grid = (double*)malloc(sizeof(double) * 2 * NN);
        double* tmp = (double*)malloc(sizeof(double) * 2 * NN);
        double* img = (double*)malloc(sizeof(double) * 2 * NN * P);
        if (!grid || !tmp || !img) {
            free(grid); free(tmp); free(img);
#ifdef _OPENMP
#pragma omp atomic write
#endif
            nomem = 1;
            continue;
        }
        double* acc = out + (size_t)c * NPP * NN;
        memset(acc, 0, sizeof(double) * NPP * NN);
        const double* taps_c = taps + (size_t)c * A * P * K * K * 2;
        const int32_t* cell_c = cell + (size_t)c * A * 2;
        for (int64_t t = 0; t < T; ++t) {
            const uint8_t* row = samples + ((size_t)t * C + c) * (size_t)A * P;
            for (int p = 0; p < P; ++p) {
                ora_grid(s, taps_c, cell_c, row, p, grid);
                dft2(N, tw, grid, tmp, img + (size_t)p * 2 * NN);
            }
            for (size_t q = 0; q < NN; ++q) {
                double xr = img[2 * q], xi = img[2 * q + 1];
                acc[q] += xr * xr + xi * xi;                       /* XX* */
                if (P == 2) {
                    double yr = img[2 * NN + 2 * q], yi = img[2 * NN + 2 * q + 1];
                    acc[NN + q] += yr * yr + yi * yi;              /* YY* */
                    acc[2 * NN + q] += xr * yr + xi * yi;          /* Re X Y* */
                    acc[3 * NN + q] += xi * yr - xr * yi;          /* Im X Y* */
                }
            }
        }
        free(grid); free(tmp); free(img);
    }
    free(cell); free(g); free(taps); free(tw);
    return nomem ? ORA_E_NOMEM : ORA_OK;
}

/* ---- the a = b terms of step 4: autocorrelation image ------------------ */
/*
 * The image of Eq. 4 is a sum over antenna pairs (a, b) (Eq. 3); this returns
 * only the pairs a = b, i.e. for every antenna its own contribution
 *   sum_t (K^p_a E^p_a(t)) (K^q_a E^q_a(t))^*  =  K^p_a K^q_a^*  sum_t E^p_a E^q_a^*
 * where K^p_a(i, j) is antenna a's kernel (with the (-1)^(x+y) factor)
 * transformed on its own, sum over taps of w (-1)^(x+y) exp(+2 pi i (x i + y j)/N).
 * The image with the autocorrelations removed is the full image minus this.
 * Same layout, channel range and threading as ora_image_range.
 */
int ora_autocorr_range(const ora_array* s, const uint8_t* samples, int64_t T,
                       int chan_begin, int chan_end, double* out, int n_threads) {
    int rc = check_array(s);
    if (rc) return rc;
    if (!samples || !out || T < 0) return ORA_E_ARG;
    if (chan_begin < 0 || chan_end > s->n_chan || chan_begin > chan_end) return ORA_E_ARG;
    const int N = s->grid_n, A = s->n_ant, P = s->n_pol, C = s->n_chan, K = s->kernel_k, h = K / 2;
    const int NPP = (P == 2) ? 4 : 1;
    const size_t NN = (size_t)N * N;

    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)C * A * 2);
    double* g = (double*)malloc(sizeof(double) * (size_t)C * A * 2);
    double* taps = (double*)malloc(sizeof(double) * (size_t)C * A * P * K * K * 2);
    double* tw = (double*)malloc(sizeof(double) * 2 * N);
    if (!cell || !g || !taps || !tw) { free(cell); free(g); free(taps); free(tw); return ORA_E_NOMEM; }
    rc = ora_geometry(s, cell, g);
    if (rc == ORA_OK) rc = ora_taps(s, cell, g, taps);
    if (rc != ORA_OK) { free(cell); free(g); free(taps); free(tw); return rc; }
    twiddle_table(N, tw);

    int nomem = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int c = chan_begin; c < chan_end; ++c) {
        double* kimg = (double*)malloc(sizeof(double) * 2 * NN * P);
        if (!kimg) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            nomem = 1;
            continue;
        }
        double* acc = out + (size_t)c * NPP * NN;
        memset(acc, 0, sizeof(double) * NPP * NN);
        const double* taps_c = taps + (size_t)c * A * P * K * K * 2;
        const int32_t* cell_c = cell + (size_t)c * A * 2;
        for (int a = 0; a < A; ++a) {
            /* the antenna's zero-lag correlations over the call: XX*, YY*, XY* */
            double vxx = 0.0, vyy = 0.0, vxyr = 0.0, vxyi = 0.0;
            for (int64_t t = 0; t < T; ++t) {
                const uint8_t* row = samples + ((size_t)t * C + c) * (size_t)A * P;
                double xr, xi;
                unpack(row[a * P], s->nibble_order, &xr, &xi);
                vxx += xr * xr + xi * xi;
                if (P == 2) {
                    double yr, yi;
                    unpack(row[a * P + 1], s->nibble_order, &yr, &yi);
                    vyy += yr * yr + yi * yi;
                    vxyr += xr * yr + xi * yi;
                    vxyi += xi * yr - xr * yi;
                }
            }
            /* the antenna's kernel transform per polarisation */
            for (int p = 0; p < P; ++p) {
                const double* w = taps_c + ((size_t)a * P + p) * K * K * 2;
                double* kp = kimg + (size_t)p * 2 * NN;
                for (int j = 0; j < N; ++j)
                    for (int i = 0; i < N; ++i) {
                        double kr = 0.0, ki = 0.0;
                        for (int dy = -h; dy <= h; ++dy)
                            for (int dx = -h; dx <= h; ++dx) {
                                int x = cell_c[2 * a + 0] + dx, y = cell_c[2 * a + 1] + dy;
                                double sgn = ((x + y) & 1) ? -1.0 : 1.0;
                                double wr = sgn * w[((dy + h) * K + (dx + h)) * 2 + 0];
                                double wi = sgn * w[((dy + h) * K + (dx + h)) * 2 + 1];
                                const double* e = tw + 2 * (((long)x * i + (long)y * j) % N);
                                kr += wr * e[0] - wi * e[1];
                                ki += wr * e[1] + wi * e[0];
                            }
                        kp[(j * N + i) * 2] = kr;
                        kp[(j * N + i) * 2 + 1] = ki;
                    }
            }
            for (size_t q = 0; q < NN; ++q) {
                double ar = kimg[2 * q], ai = kimg[2 * q + 1];
                acc[q] += vxx * (ar * ar + ai * ai);                         /* XX* */
                if (P == 2) {
                    double br = kimg[2 * NN + 2 * q], bi = kimg[2 * NN + 2 * q + 1];
                    acc[NN + q] += vyy * (br * br + bi * bi);                /* YY* */
                    /* K^X K^Y* times the correlation X Y* */
                    double kr = ar * br + ai * bi, ki = ai * br - ar * bi;
                    acc[2 * NN + q] += vxyr * kr - vxyi * ki;                /* Re X Y* */
                    acc[3 * NN + q] += vxyr * ki + vxyi * kr;                /* Im X Y* */
                }
            }
        }
        free(kimg);
    }
    free(cell); free(g); free(taps); free(tw);
    return nomem ? ORA_E_NOMEM : ORA_OK;
}

/* ---- steps 1-3 only: electric-field images ------------------------------ */
/*
 * out: FP64 [T][C][P][N][N][2] (overwritten for the channel range): for every
 * spectrum the transformed field of step 3 of each polarisation, before the
 * products of step 4.  Same arguments as ora_image_range otherwise.
 */
int ora_efield_range(const ora_array* s, const uint8_t* samples, int64_t T,
                     int chan_begin, int chan_end, double* out, int n_threads) {
    int rc = check_array(s);
    if (rc) return rc;
    if (!samples || !out || T < 0) return ORA_E_ARG;
    if (chan_begin < 0 || chan_end > s->n_chan || chan_begin > chan_end) return ORA_E_ARG;
    const int N = s->grid_n, A = s->n_ant, P = s->n_pol, C = s->n_chan, K = s->kernel_k;
    const size_t NN = (size_t)N * N;

    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)C * A * 2);
    double* g = (double*)malloc(sizeof(double) * (size_t)C * A * 2);
    double* taps = (double*)malloc(sizeof(double) * (size_t)C * A * P * K * K * 2);
    double* tw = (double*)malloc(sizeof(double) * 2 * N);
    if (!cell || !g || !taps || !tw) { free(cell); free(g); free(taps); free(tw); return ORA_E_NOMEM; }
    rc = ora_geometry(s, cell, g);
    if (rc == ORA_OK) rc = ora_taps(s, cell, g, taps);
    if (rc != ORA_OK) { free(cell); free(g); free(taps); free(tw); return rc; }
    twiddle_table(N, tw);

    int nomem = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int c = chan_begin; c < chan_end; ++c) {
        double* grid = (double*)malloc(sizeof(double) * 2 * NN);
        double* tmp = (double*)malloc(sizeof(double) * 2 * NN);
        if (!grid || !tmp) {
            free(grid); free(tmp);
#ifdef _OPENMP
#pragma omp atomic write
#endif
            nomem = 1;
            continue;
        }
        const double* taps_c = taps + (size_t)c * A * P * K * K * 2;
        const int32_t* cell_c = cell + (size_t)c * A * 2;
        for (int64_t t = 0; t < T; ++t) {
            const uint8_t* row = samples + ((size_t)t * C + c) * (size_t)A * P;
            for (int p = 0; p < P; ++p) {
                ora_grid(s, taps_c, cell_c, row, p, grid);
                dft2(N, tw, grid, tmp, out + (((size_t)t * C + c) * P + p) * 2 * NN);
            }
        }
        free(grid); free(tmp);
    }
    free(cell); free(g); free(taps); free(tw);
    return nomem ? ORA_E_NOMEM : ORA_OK;
}

int ora_image(const ora_array* s, const uint8_t* samples, int64_t T, double* out, int n_threads) {
    if (!s) return ORA_E_ARG;
    return ora_image_range(s, samples, T, 0, s->n_chan, out, n_threads);
}

int ora_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
