"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each compares it with an
independent route (FX correlation, a library FFT, a closed form, an identity,
an exhaustive table) chosen so that a dropped term, a wrong sign or index, or a
transposed operand fails at least one of them.  ``test_planted_mistakes``
checks exactly that by compiling mutated copies of the oracle source.
"""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import synth
from fx_bruteforce import fx_image, kernel_images, unpack_int

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


class Sub:
    """Minimal sub-array description for hand-built cases."""

    def __init__(self, xy, n_pol=1, n_chan=1, grid_n=32, grid_dl=0.5, f0=40e6, df=25e3, k=3):
        self.ant_xy = np.asarray(xy, dtype=np.float64)
        self.n_pol, self.n_chan, self.grid_n, self.grid_dl = n_pol, n_chan, grid_n, grid_dl
        self.freq0_hz, self.dfreq_hz, self.kernel_k = f0, df, k


# ---------------------------------------------------------------- unpack
@pytest.mark.parametrize("order", [0, 1])
def test_unpack_exhaustive(order):
    """All 256 codes against two's-complement nibbles taken by int8 shifts."""
    re, im = oracle.unpack_table(order)
    codes = np.arange(256, dtype=np.uint8)
    r2, i2 = unpack_int(codes, order)
    assert np.array_equal(re, r2.astype(float)) and np.array_equal(im, i2.astype(float))
    assert re.min() == -8 and re.max() == 7
    # spot values of the encoding: 0x7F -> (7, -1), 0x80 -> (-8, 0), 0x08 -> (0, -8)
    if order == 0:
        assert (re[0x7F], im[0x7F]) == (7, -1)
        assert (re[0x80], im[0x80]) == (-8, 0)
        assert (re[0x08], im[0x08]) == (0, -8)


# ---------------------------------------------------------------- geometry
def test_geometry_special_cases():
    """lambda = 1 m (f = c0), dl = 0.5: an antenna at x metres sits at cell
    N/2 + 2x; the origin is the centre; half-cell ties round up."""
    xs = [0.0, 0.5, -0.5, 3.0, -4.0, 0.25, -0.25, 0.75]
    xy = [[x, -x] for x in xs]
    s = Sub(xy, grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0)
    cell, g = oracle.geometry(s)
    expect_g = np.array([[16 + 2 * x, 16 - 2 * x] for x in xs])
    assert np.array_equal(g[0], expect_g)
    # ties: 16.5 -> 17, 15.5 -> 16, 17.5 -> 18, 14.5 -> 15
    exp_cell = [[16, 16], [17, 15], [15, 17], [22, 10], [8, 24], [17, 16], [16, 17], [18, 15]]
    assert cell[0].tolist() == exp_cell


def test_geometry_scales_with_frequency():
    """Cell offsets from the centre are x f / (c0 dl): doubling f doubles them."""
    s = Sub([[3.0, -2.0], [-5.0, 1.5]], n_chan=2, grid_n=64, grid_dl=1.0, f0=30e6, df=30e6)
    _, g = oracle.geometry(s)
    off = g - 32.0
    np.testing.assert_allclose(off[1], 2.0 * off[0], rtol=1e-12)
    lam0 = 299792458.0 / 30e6
    np.testing.assert_allclose(off[0], np.array([[3.0, -2.0], [-5.0, 1.5]]) / lam0, rtol=1e-12)


def test_geometry_out_of_grid():
    s = Sub([[0.0, 0.0], [7.4, 0.0]], grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0)
    # 7.4 m -> g = 30.8 -> cell 31 -> footprint reaches 32 > N-1
    with pytest.raises(oracle.OracleError) as e:
        oracle.geometry(s)
    assert e.value.code == oracle.ORA_E_GEOMETRY


def test_geometry_footprint_grows_with_kernel_size():
    """The footprint is the K x K block centred on the nearest cell: an
    antenna at cell 29 of a 32-cell grid fits with K = 3 and 5 (cells 27..31)
    but not with K = 7 (26..32); one at cell 2 fits K = 5 but not K = 7."""
    for xs, ok in (([6.4], (1, 3, 5)), ([-7.0], (1, 3, 5))):
        for k in (1, 3, 5, 7):
            s = Sub([[x, 0.0] for x in xs], grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0, k=k)
            if k in ok:
                cell, _ = oracle.geometry(s)
                assert cell[0, 0, 0] in (29, 2)
            else:
                with pytest.raises(oracle.OracleError) as e:
                    oracle.geometry(s)
                assert e.value.code == oracle.ORA_E_GEOMETRY


# ---------------------------------------------------------------- taps
def _gauss_1d(p0, g, k, sigma):
    """Normalised 1-D Gaussian weights of the k cells p0 - k/2 .. p0 + k/2 at
    the antenna coordinate g."""
    d = p0 + np.arange(-(k // 2), k // 2 + 1) - g
    w = np.exp(-d * d / (2.0 * sigma * sigma))
    return w / w.sum()


@pytest.mark.parametrize("k", [1, 3, 5, 7])
@pytest.mark.parametrize("sigma", [0.35, 0.5, 0.8])
def test_gaussian_taps_separable_closed_form(k, sigma):
    """Any odd K and sigma.  exp(-(ex^2 + ey^2) / (2 s^2)) is the product of a
    Gaussian in ex and one in ey, and the K x K tap block is the product set
    of its rows and columns, so the normalised kernel is the outer product of
    two 1-D Gaussians, each normalised on its own.  At zero sub-cell offset
    both are exp(-d^2 / (2 s^2)), d = -K/2..K/2, over their sum; K = 1 is a
    single tap of weight 1."""
    lam = 1.0                                           # f = c0: one metre per wavelength
    xy = [[0.0, 0.0], [0.3, -0.45], [-1.2, 2.7]]        # dl = 0.5: two cells per metre
    s = Sub(xy, n_pol=2, grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0, k=k)
    tp = oracle.taps(s, kernel_sigma_cells=sigma)
    assert tp.shape == (1, 3, 2, k, k)
    assert np.all(tp.imag == 0)
    d = np.arange(-(k // 2), k // 2 + 1, dtype=float)
    w0 = np.exp(-d * d / (2.0 * sigma * sigma))
    w0 /= w0.sum()
    np.testing.assert_allclose(tp[0, 0, 0].real, np.outer(w0, w0), rtol=0, atol=1e-15)
    if k == 1:
        assert np.all(tp.real == 1.0)
    for a, (x, y) in enumerate(xy):
        gx, gy = 16 + 2 * x / lam, 16 + 2 * y / lam
        px, py = np.floor(gx + 0.5), np.floor(gy + 0.5)
        expect = np.outer(_gauss_1d(py, gy, k, sigma), _gauss_1d(px, gx, k, sigma))
        for p in range(2):   # the same kernel for both pols
            np.testing.assert_allclose(tp[0, a, p].real, expect, rtol=1e-13, atol=1e-16)


def test_gaussian_sigma_sets_the_tap_ratio():
    """At zero offset the ratio of the centre tap to its neighbour is
    exp(1 / (2 s^2)) for any K: sigma enters squared, in the denominator."""
    for k in (3, 5, 7):
        for sigma in (0.35, 0.8, 1.5):
            s = Sub([[0.0, 0.0]], grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0, k=k)
            row = oracle.taps(s, kernel_sigma_cells=sigma)[0, 0, 0].real[k // 2]
            c = k // 2
            np.testing.assert_allclose(row[c] / row[c + 1], np.exp(1.0 / (2 * sigma * sigma)), rtol=1e-13)
            if k > 3:   # distances 1 -> 2: exp((4 - 1) / (2 s^2))
                np.testing.assert_allclose(row[c + 1] / row[c + 2], np.exp(3.0 / (2 * sigma * sigma)), rtol=1e-13)


def test_gaussian_taps_closed_form():
    """Zero sub-cell offset, sigma = 0.5 cell: the 3x3 kernel is the outer
    product of [e^-2, 1, e^-2] / (1 + 2 e^-2) with itself."""
    s = Sub([[0.0, 0.0], [1.0, -0.5]], grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0)
    tp = oracle.taps(s)
    w1 = np.array([np.exp(-2.0), 1.0, np.exp(-2.0)]) / (1.0 + 2.0 * np.exp(-2.0))
    np.testing.assert_allclose(tp[0, 0, 0].real, np.outer(w1, w1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(tp[0, :, 0].sum(axis=(-1, -2)), 1.0, rtol=0, atol=1e-14)
    assert np.all(tp.imag == 0)


def test_gaussian_taps_follow_offset():
    """An antenna a quarter cell right of a cell centre weights its right
    neighbour more than its left one, by exp((d_l^2 - d_r^2) / (2 s^2))."""
    # g = 16.25: cell 16, taps at 15, 16, 17 are at distances 1.25, 0.25, 0.75
    s = Sub([[0.125, 0.0]], grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0)
    tp = oracle.taps(s)[0, 0, 0].real
    row = tp[1]  # dy = 0
    np.testing.assert_allclose(row[2] / row[0], np.exp((1.25 ** 2 - 0.75 ** 2) / 0.5), rtol=1e-13)


def test_user_taps_pass_through():
    s = Sub([[0.0, 0.0]], n_pol=2, grid_n=32, grid_dl=0.5, f0=299792458.0, df=0.0)
    rng = np.random.default_rng(3)
    t = rng.standard_normal((1, 1, 2, 3, 3, 2)).astype(np.float32)
    tp = oracle.taps(s, taps=t)
    np.testing.assert_array_equal(tp, t[..., 0].astype(np.float64) + 1j * t[..., 1].astype(np.float64))


# ---------------------------------------------------------------- DFT
@pytest.mark.parametrize("n", [8, 12, 32, 48])
def test_dft_is_library_inverse_fft(n):
    """The unnormalised exp(+...) DFT equals numpy's ifft2 times N^2."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    np.testing.assert_allclose(oracle.dft2(x), np.fft.ifft2(x) * n * n, rtol=0, atol=1e-11 * n * n)


def test_dft_orientation():
    """A single cell at (x=1, y=0) gives exp(+2 pi i i/N) varying along i only."""
    n = 16
    x = np.zeros((n, n), complex)
    x[0, 1] = 1.0
    d = oracle.dft2(x)
    i = np.arange(n)
    np.testing.assert_allclose(d, np.tile(np.exp(2j * np.pi * i / n), (n, 1)), atol=1e-14)


# ---------------------------------------------------------------- worked example
def _on_grid_example(n_ant, grid_n, axis, T=3, seed=11):
    """Antennas on cell centres (lambda = 1 m, dl = 0.5); a real source of
    amplitude 7 at l0 = 1/(4 dl) (axis 0) or m0 = 1/(4 dl) (axis 1).  Phases are
    multiples of pi/2 so every sample is exactly 4-bit: 7 (-i)^n."""
    rng = np.random.default_rng(seed)
    lim = grid_n // 2 - 3
    pos = set()
    while len(pos) < n_ant:
        pos.add((int(rng.integers(-lim, lim + 1)), int(rng.integers(-lim, lim + 1))))
    cells = np.array(sorted(pos))
    xy = cells * 0.5                       # metres: offset of n cells = n * dl * lambda
    s = Sub(xy, grid_n=grid_n, grid_dl=0.5, f0=299792458.0, df=0.0)
    nsteps = cells[:, axis]                # u l0 = n/4 -> phase -pi n / 2
    ph = (-1j) ** (nsteps % 4)
    e = 7 * ph
    b = synth.pack44(np.rint(e.real).astype(int), np.rint(e.imag).astype(int))
    samples = np.broadcast_to(b[None, None, :, None], (T, 1, n_ant, 1)).copy()
    return s, samples


@pytest.mark.parametrize("axis", [0, 1])
def test_worked_example_closed_form(axis):
    """Peak value T (7 A w0)^2 with w0 = 1/(1 + 2 e^-2) (the centre of the 1-D
    normalised kernel), at pixel (j, i) = (N/2, 3N/4) for a source along l and
    (3N/4, N/2) along m; checked against the committed golden values."""
    A, N, T = 10, 32, 3
    s, x = _on_grid_example(A, N, axis, T)
    img = oracle.image(s, x)[0, 0]
    w0 = 1.0 / (1.0 + 2.0 * np.exp(-2.0))
    peak = T * (7.0 * A * w0) ** 2
    jj, ii = np.unravel_index(np.argmax(img), img.shape)
    assert (jj, ii) == ((N // 2, 3 * N // 4) if axis == 0 else (3 * N // 4, N // 2))
    assert abs(img[jj, ii] - peak) <= 1e-12 * peak
    gold = dict(l.split("=") for l in open(os.path.join(GOLDEN, "worked_example.txt")).read().split()
                if "=" in l)
    assert abs(peak / T - float(gold["peak_per_sample_A10"])) < 1e-6


# ---------------------------------------------------------------- identities
def test_fx_identity_tiny_config():
    """Config-1 shape: oracle image == FX correlation + direct imaging (Eq. 3)."""
    sub = synth.workload(1).subs[0]
    x = synth.samples(sub, 64)
    img = oracle.image(sub, x)
    cell, _ = oracle.geometry(sub)
    ref = fx_image(x, cell, oracle.taps(sub), sub.grid_n)
    assert np.abs(img - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fx_identity_dual_pol_user_taps():
    """Dual pol, complex per-pol user taps, station layout subset."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=48)
    x = synth.samples(sub, 24)
    rng = np.random.default_rng(5)
    t = rng.standard_normal((2, 48, 2, 3, 3, 2)).astype(np.float32)
    img = oracle.image(sub, x, taps=t)
    cell, _ = oracle.geometry(sub)
    ref = fx_image(x, cell, oracle.taps(sub, taps=t), sub.grid_n)
    scale = np.sqrt(np.abs(ref[:, 0]).max() * np.abs(ref[:, 1]).max())
    assert np.abs(img - ref).max() <= 1e-12 * scale


def test_autocorr_removed_is_fx_without_diagonal():
    """Image with the autocorrelations removed == FX imaging of the a != b
    baselines only (dual pol, complex per-pol user taps)."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=40)
    x = synth.samples(sub, 20)
    rng = np.random.default_rng(6)
    t = rng.standard_normal((2, 40, 2, 3, 3, 2)).astype(np.float32)
    img = oracle.image(sub, x, taps=t, remove_autocorr=True)
    cell, _ = oracle.geometry(sub)
    ref = fx_image(x, cell, oracle.taps(sub, taps=t), sub.grid_n, drop_auto=True)
    full = fx_image(x, cell, oracle.taps(sub, taps=t), sub.grid_n)
    scale = np.sqrt(np.abs(full[:, 0]).max() * np.abs(full[:, 1]).max())
    assert np.abs(img - ref).max() <= 1e-12 * scale


def test_autocorr_is_sum_of_single_antenna_images():
    """The a = b image equals the sum of the images of one-antenna arrays
    (each antenna keeps its own cell and taps), by the main imaging route."""
    import copy
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=6)
    x = synth.samples(sub, 16)
    au = oracle.autocorr(sub, x)
    tot = np.zeros_like(au)
    for a in range(sub.n_ant):
        one = copy.copy(sub)
        one.ant_xy = sub.ant_xy[a:a + 1]   # n_ant follows ant_xy
        tot += oracle.image(one, np.ascontiguousarray(x[:, :, a:a + 1]))
    assert np.abs(au - tot).max() <= 1e-12 * np.abs(tot).max()
    # the single-pol tiny configuration too
    sub1 = synth.workload(1).subs[0]
    x1 = synth.samples(sub1, 32)
    cell, _ = oracle.geometry(sub1)
    ref = fx_image(x1, cell, oracle.taps(sub1), sub1.grid_n) - fx_image(x1, cell, oracle.taps(sub1), sub1.grid_n,
                                                                          drop_auto=True)
    assert np.abs(oracle.autocorr(sub1, x1) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_efield_single_antenna_is_kernel_image():
    """One antenna: its field image is E times its kernel transform K(i, j),
    evaluated directly per pixel (independent of the gridding + DFT route)."""
    import copy
    sub = copy.copy(synth.shrink(synth.workload(2).subs[0], n_chan=2))
    sub.ant_xy = sub.ant_xy[5:6]
    x = synth.samples(synth.shrink(synth.workload(2).subs[0], n_chan=2), 3)[:, :, 5:6]
    x = np.ascontiguousarray(x)
    ef = oracle.efield(sub, x)
    cell, _ = oracle.geometry(sub)
    re, im = unpack_int(x)
    for c in range(2):
        kimg = kernel_images(cell[c], oracle.taps(sub)[c], sub.grid_n)   # [A=1][P][j][i]
        for t in range(3):
            for p in range(2):
                e = re[t, c, 0, p] + 1j * im[t, c, 0, p]
                assert np.abs(ef[t, c, p] - e * kimg[0, p]).max() <= 1e-12 * (np.abs(kimg[0, p]).max() * 12)


def test_efield_products_sum_to_image():
    """Summed over spectra, |X|^2, |Y|^2 and X Y* of the field images are the
    four products of the (FX-pinned) image."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=32)
    x = synth.samples(sub, 7)
    ef = oracle.efield(sub, x)
    img = oracle.image(sub, x)
    X, Y = ef[:, :, 0], ef[:, :, 1]
    ref = np.stack([(np.abs(X) ** 2).sum(0), (np.abs(Y) ** 2).sum(0), (X * np.conj(Y)).real.sum(0),
                    (X * np.conj(Y)).imag.sum(0)], axis=1)
    assert np.abs(img - ref).max() <= 1e-12 * np.abs(img).max()


def test_parseval():
    """sum_pixels XX* = N^2 sum_t sum_cells |G_X|^2, and the same for X Y*."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=1, n_ant=40)
    x = synth.samples(sub, 5)
    img = oracle.image(sub, x)
    N = sub.grid_n
    gx = [oracle.grid(sub, x, t, 0, 0) for t in range(5)]
    gy = [oracle.grid(sub, x, t, 0, 1) for t in range(5)]
    ex = N * N * sum((np.abs(g) ** 2).sum() for g in gx)
    exy = N * N * sum((a * np.conj(b)).sum() for a, b in zip(gx, gy))
    assert abs(img[0, 0].sum() - ex) <= 1e-12 * ex
    assert abs(img[0, 2].sum() - exy.real) <= 1e-12 * ex
    assert abs(img[0, 3].sum() - exy.imag) <= 1e-12 * ex


def test_polarisation_conjugation_order():
    """Y = i X on every antenna gives Re XY* = 0 and Im XY* = -XX* exactly, so the
    phase of XY* at a source is -psi for Y = e^{i psi} X (psi = pi/2 here)."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=32)
    x = synth.samples(sub, 6)
    re, im = unpack_int(x[..., 0])
    # Y = i X: (re, im) -> (-im, re); -(-8) is out of range, clip those to 7
    yr = np.clip(-im, -8, 7)
    ok = yr == -im
    xr, xi = np.where(ok, re, 0), np.where(ok, im, 0)
    bx = synth.pack44(xr, xi)
    by = synth.pack44(-xi, xr)
    xx = np.stack([bx, by], axis=-1)
    img = oracle.image(sub, xx)
    assert np.all(img[:, 2] == 0.0)
    assert np.array_equal(img[:, 3], -img[:, 0])
    assert np.array_equal(img[:, 1], img[:, 0])


def test_invariants_and_linearity():
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=64)
    x = synth.samples(sub, 16)
    img = oracle.image(sub, x)
    xx, yy, xr, xi = img[:, 0], img[:, 1], img[:, 2], img[:, 3]
    assert (xx >= 0).all() and (yy >= 0).all()
    assert (xr ** 2 + xi ** 2 <= xx * yy * (1 + 1e-12) + 1e-9).all()         # Cauchy-Schwarz
    half = oracle.image(sub, x[:8]) + oracle.image(sub, x[8:])
    assert np.abs(half - img).max() <= 1e-12 * np.abs(img).max()
    zero = np.zeros_like(x)
    assert not oracle.image(sub, zero).any()
    # empty call: no spectra, all-zero image
    assert not oracle.image(sub, x[:0]).any()


def test_point_source_localisation():
    """A noisy point source peaks at its predicted pixel once the image is
    divided by the kernel beam sum_a |K_a|^2 (the A(l, m) of Eq. 1)."""
    from fx_bruteforce import kernel_images
    sub = synth.workload(1).subs[0]
    N = sub.grid_n
    for k, (i0, j0) in enumerate([(16, 16), (19, 13), (12, 20)]):
        s = synth.shrink(sub, n_chan=2)
        s.sources = [synth.Source(i0, j0, 2.0)]
        s.seed_key = (synth.ROOT_SEED, 99, k)
        x = synth.samples(s, 256)
        img = oracle.image(s, x)
        cell, _ = oracle.geometry(s)
        tp = oracle.taps(s)
        for c in range(2):
            beam = (np.abs(kernel_images(cell[c], tp[c], N)[:, 0]) ** 2).sum(axis=0)
            jj, ii = np.unravel_index(np.argmax(img[c, 0] / beam), (N, N))
            assert (ii, jj) == (i0, j0)


# ---------------------------------------------------------------- mutations
MUTANTS = {
    # dropped term: the last antenna never reaches the grid
    "drop_antenna": ("for (int a = 0; a < A; ++a) {\n        double er, ei;",
                     "for (int a = 0; a < A - 1; ++a) {\n        double er, ei;"),
    # wrong sign of the transform
    "dft_sign": ("tw[2 * r + 1] = sin(", "tw[2 * r + 1] = -sin("),
    # transposed operand: rows and columns swapped when writing the row pass
    "transpose": ("tmp[(y * N + i) * 2] = ar;\n            tmp[(y * N + i) * 2 + 1] = ai;",
                  "tmp[(i * N + y) * 2] = ar;\n            tmp[(i * N + y) * 2 + 1] = ai;"),
    # conjugate on the wrong factor of XY*
    "conj_order": ("acc[3 * NN + q] += xi * yr - xr * yi;", "acc[3 * NN + q] += xr * yi - xi * yr;"),
    # nibble order swapped
    "nibble": ("if (order == 0) { *re = hi; *im = lo; }", "if (order == 0) { *re = lo; *im = hi; }"),
    # checkerboard dropped
    "checkerboard": ("double sgn = ((x + y) & 1) ? -1.0 : 1.0;\n                double wr = w[",
                     "double sgn = 1.0;\n                double wr = w["),
    # autocorrelation image: checkerboard dropped from the lone kernel transform
    "auto_checkerboard": ("double sgn = ((x + y) & 1) ? -1.0 : 1.0;\n                                double wr = sgn",
                          "double sgn = 1.0;\n                                double wr = sgn"),
    # autocorrelation image: conjugate on the wrong factor of the correlation X Y*
    "auto_conj": ("vxyi += xi * yr - xr * yi;", "vxyi += xr * yi - xi * yr;"),
    # autocorrelation image: kernel cross term without the conjugate
    "auto_kernel_conj": ("double kr = ar * br + ai * bi, ki = ai * br - ar * bi;",
                         "double kr = ar * br - ai * bi, ki = ai * br + ar * bi;"),
    # Gaussian not normalised
    "no_norm": ("for (int k = 0; k < K * K; ++k) w[2 * k] /= sum;", "(void)sum;"),
    # rounding to nearest cell replaced by truncation
    "floor": ("double p = floor(gg + 0.5);", "double p = floor(gg);"),
    # kernel half-width hard-coded to 1 (right only for K = 3)
    "taps_half_width": ("const int A = s->n_ant, P = s->n_pol, K = s->kernel_k, h = K / 2;",
                        "const int A = s->n_ant, P = s->n_pol, K = s->kernel_k, h = 1;"),
    # footprint check with the half-width hard-coded to 1
    "geometry_half_width": ("const int N = s->grid_n, h = s->kernel_k / 2;", "const int N = s->grid_n, h = 1;"),
    # sigma ignored (the default 0.5 always)
    "sigma_fixed": ("double sig = s->kernel_sigma_cells > 0.0 ? s->kernel_sigma_cells : 0.5;",
                    "double sig = 0.5;"),
}


def _pins_pass() -> bool:
    try:
        test_unpack_exhaustive(0)
        test_geometry_special_cases()
        test_gaussian_taps_closed_form()
        test_gaussian_taps_separable_closed_form(5, 0.8)
        test_gaussian_taps_separable_closed_form(7, 0.35)
        test_geometry_footprint_grows_with_kernel_size()
        for ax in (0, 1):
            test_worked_example_closed_form(ax)
        test_fx_identity_dual_pol_user_taps()
        test_autocorr_removed_is_fx_without_diagonal()
        test_polarisation_conjugation_order()
        test_dft_orientation()
    except (AssertionError, oracle.OracleError, pytest.fail.Exception):
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes(name, tmp_path):
    """Each planted mistake in a copy of the oracle source fails some pin."""
    src = open(oracle.source_path()).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    mut = tmp_path / f"m_{name}.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / f"libm_{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    str(mut), "-o", str(lib), "-lm"], check=True)
    with oracle.using_library(str(lib)):
        assert not _pins_pass(), f"mutant {name} passed every pin"
    assert _pins_pass()
