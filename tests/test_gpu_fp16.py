"""GPU parity of the FP16 matrix-core form against the FP64 oracle.

Tolerance 1e-3 per image (relative Frobenius error and max |diff| over the
channel peak), the bar for the reduced-precision forms.  The FP16 operands
are the gridded aperture (4-bit samples times FP32 weights), the row-pass
output and the DFT matrix; each adds ~2^-12 relative rounding, which a CPU
simulation of the same arithmetic puts at ~1.2e-4 per image for the station
layout, so 1e-3 leaves a margin of ~8.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_parity, check_invariants, image_errors, oracle_channels, run_library

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def test_station_subset(E):
    sub = synth.shrink(synth.workload(3).subs[0], n_chan=5)
    x = synth.samples(sub, 40)
    (gpu,), info = run_library(E, [sub], [x], precision="fp16")
    assert info["precision"] == E.EPIC_FP16
    fro, mx = assert_parity(gpu, oracle.image(sub, x), TOL, "cfg3-subset")
    print(f"fp16 station subset: max per-image rel err {fro:.2e}, max |d|/peak {mx:.2e}")


@pytest.mark.parametrize("cfg,k,nchan,T", [(4, 0, 2, 12), (4, 1, 3, 12), (4, 2, 2, 8), (5, 0, 1, 4), (1, 0, 4, 64)])
def test_other_shapes(E, cfg, k, nchan, T):
    """N = 64, 48, 96 (window 48 -> 3 MFMA steps), 128 (column split) and the
    single-pol 32x32 case."""
    sub = synth.shrink(synth.workload(cfg).subs[k], n_chan=nchan)
    x = synth.samples(sub, T)
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16")
    assert_parity(gpu, oracle.image(sub, x), TOL, f"fp16 cfg{cfg}.{k}")


def test_split_calls_deterministic(E):
    sub = synth.shrink(synth.workload(3).subs[0], n_chan=3)
    x = synth.samples(sub, 21)
    (a,), _ = run_library(E, [sub], [x], precision="fp16", calls=[21])
    (b,), _ = run_library(E, [sub], [x], precision="fp16", calls=[21])
    assert np.array_equal(a, b)
    (c,), _ = run_library(E, [sub], [x], precision="fp16", calls=[10, 11])
    assert_parity(c, oracle.image(sub, x), TOL, "fp16 split")


def test_complex_user_taps(E):
    sub = synth.shrink(synth.workload(3).subs[0], n_chan=2, n_ant=64)
    x = synth.samples(sub, 12)
    taps = np.random.default_rng(4).standard_normal((2, 64, 2, 3, 3, 2)).astype(np.float32)
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16", taps=[taps])
    assert_parity(gpu, oracle.image(sub, x, taps=taps), TOL, "fp16 user taps")


def test_full_station_all_channels(E):
    """Config 3 at full size (132 channels, 1000 spectra in one call), every
    channel against the oracle; the per-channel error is reported."""
    sub, x, ora = oracle_channels(2, 1000)    # the same station and samples as config 3
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16")
    fro, mx = image_errors(gpu, ora)
    worst = np.argsort(fro.max(axis=1))[::-1][:3]
    print("cfg3 per-channel max rel err: " + ", ".join(f"c{c} {fro[c].max():.2e}" for c in worst) +
          f"; median {np.median(fro.max(axis=1)):.2e}")
    assert_parity(gpu, ora, TOL, "cfg3 full, all 132 channels")
    check_invariants(gpu)


def test_degenerate_arrays_and_swapped_nibbles(E):
    """One antenna; two antennas whose kernels touch cells 0 and N-1 (the
    window spans the whole grid); nibble order 1 -- in the FP16 form."""
    lam = 299792458.0 / 40e6

    class S:
        n_pol, n_chan, grid_n, grid_dl, freq0_hz, dfreq_hz, kernel_k = 2, 1, 32, 0.5, 40e6, 0.0, 3
    edge = np.array([[-15 * 0.5 * lam, -15 * 0.5 * lam], [14 * 0.5 * lam, 14 * 0.5 * lam]])
    for k, xy in enumerate((np.array([[1.3, -2.2]]), edge)):
        s = S()
        s.ant_xy = xy
        x = np.random.default_rng(20 + k).integers(0, 256, (7, 1, len(xy), 2), dtype=np.uint8)
        for order in (0, 1):
            (gpu,), _ = run_library(E, [s], [x], precision="fp16", nibble_order=order)
            assert_parity(gpu, oracle.image(s, x, nibble_order=order), TOL, f"fp16 edge{len(xy)} order{order}")


def test_full_large_array_sampled_channels(E):
    """The 2048-antenna array at full size (256 channels, N = 128, 125 spectra
    in one call) in the FP16 form, against the oracle on three channels."""
    chans = (0, 128, 255)
    sub, x, ora = oracle_channels(5, 125, chans)
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16")
    for c in chans:
        fro, mx = assert_parity(gpu[c:c + 1], ora[c:c + 1], TOL, f"large array fp16 full, channel {c}")
        print(f"large array fp16 channel {c}: rel err {fro:.2e}, max |d|/peak {mx:.2e}")
    check_invariants(gpu)


def test_single_pol_split_columns(E):
    """Single-pol array on a 128 grid (columns over two workgroups) in the
    FP16 form."""
    import dataclasses
    base = synth.shrink(synth.workload(2).subs[0], n_chan=2)
    sub = dataclasses.replace(base, n_pol=1, grid_n=128, grid_dl=1.0)
    x = synth.samples(sub, 5)
    (gpu,), info = run_library(E, [sub], [x], precision="fp16")
    assert info["col_split"][0] == 2 and info["npp"][0] == 1
    assert_parity(gpu, oracle.image(sub, x), TOL, "fp16 single pol N=128")


@pytest.mark.parametrize("n,dl,nchan,T,ks", [(256, 0.5, 2, 3, 8), (192, 0.5, 1, 4, 4)])
def test_wide_grids(E, n, dl, nchan, T, ks):
    """256 x 256 (image columns over eight workgroups, 16 row waves each) and
    192 x 192 (four) in the FP16 form, station layout at half-wavelength cells."""
    import dataclasses
    sub = dataclasses.replace(synth.shrink(synth.workload(2).subs[0], n_chan=nchan), grid_n=n, grid_dl=dl)
    x = synth.samples(sub, T)
    (gpu,), info = run_library(E, [sub], [x], precision="fp16")
    assert info["col_split"][0] == ks and info["threads"][0] == 64 * n // 16
    fro, mx = assert_parity(gpu, oracle.image(sub, x), TOL, f"fp16 N={n}")
    print(f"fp16 N={n}: rel err {fro:.2e}, max |d|/peak {mx:.2e}")


def test_full_wide_grid_sampled_channel(E):
    """The station on a 256 x 256 grid at half-wavelength cells (132 channels,
    100 spectra in one call) in the FP16 form, against the oracle on its
    highest channel (the largest window); invariants on all channels."""
    sub, x, ora = oracle_channels(6, 100, (131,))
    (gpu,), info = run_library(E, [sub], [x], precision="fp16")
    assert info["col_split"][0] == 8
    fro, mx = assert_parity(gpu[131:132], ora[131:132], TOL, "fp16 256 grid full, channel 131")
    print(f"fp16 256 grid full, channel 131: rel err {fro:.2e}, max |d|/peak {mx:.2e}")
    check_invariants(gpu)
