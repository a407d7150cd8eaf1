"""Integration checks of the GPU images that do not go through the oracle's
values: a noisy point source peaks at its predicted pixel (after dividing by
the kernel beam, the A(l, m) of Eq. 1), in the FP32 and FP16 forms."""
import numpy as np
import pytest

import oracle
import synth
from fx_bruteforce import kernel_images
from gpu_util import run_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_point_source_at_predicted_pixel(E, precision):
    sub = synth.workload(1).subs[0]
    N = sub.grid_n
    for k, (i0, j0) in enumerate([(16, 16), (19, 13), (12, 20)]):
        s = synth.shrink(sub, n_chan=2)
        s.sources = [synth.Source(i0, j0, 2.0)]
        s.seed_key = (synth.ROOT_SEED, 99, k)
        x = synth.samples(s, 256)
        (img,), _ = run_library(E, [s], [x], precision=precision)
        cell, _ = oracle.geometry(s)
        tp = oracle.taps(s)
        for c in range(2):
            beam = (np.abs(kernel_images(cell[c], tp[c], N)[:, 0]) ** 2).sum(axis=0)
            jj, ii = np.unravel_index(np.argmax(img[c, 0] / beam), (N, N))
            assert (ii, jj) == (i0, j0), f"{precision}: source at {(i0, j0)}, peak at {(ii, jj)}"


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 1e-3)])
def test_polarisation_convention(E, precision, tol):
    """Y = i X on every antenna: XY* = -i |X|^2, so Re XY* vanishes, Im XY*
    equals -XX* and YY* equals XX* in every pixel (up to rounding), which pins
    the conjugated factor of the cross product."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=32)
    x = synth.samples(sub, 6)
    b = x[..., 0].astype(np.int64)
    re, im = ((b >> 4) ^ 8) - 8, ((b & 15) ^ 8) - 8
    ok = -im <= 7                                   # -(-8) does not fit a nibble
    xr, xi = np.where(ok, re, 0), np.where(ok, im, 0)
    bx = synth.pack44(xr, xi)
    by = synth.pack44(-xi, xr)
    xx = np.ascontiguousarray(np.stack([bx, by], axis=-1))
    (img,), _ = run_library(E, [sub], [xx], precision=precision)
    for c in range(sub.n_chan):
        peak = img[c, 0].max()
        assert np.abs(img[c, 2]).max() <= tol * peak
        assert np.abs(img[c, 3] + img[c, 0]).max() <= tol * peak
        assert np.abs(img[c, 1] - img[c, 0]).max() <= tol * peak
