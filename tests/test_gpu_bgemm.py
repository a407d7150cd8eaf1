"""Gridding on the matrix cores (EPIC_GRID_BLOCK_GEMM, EPIC_GRID_DENSE_GEMM),
FP16 and FP8 operands, against the FP64 oracle.

The gridding step (Eq. 4: every antenna's field through its kernel, summed
over antennas) runs as the product of the channel's kernel matrix with the
spectra's fields; the transforms and products are those of the FP16 form.
Bar: 1e-3 per image (the reduced-precision bar).  FP16 weights are split
hi + lo (~2^-22 relative), FP8 weights are a scaled e4m3 hi + lo pair
(<= 2^-8 relative per weight); the 4-bit samples are exact in both, and the
transform stages round like the FP16 gather form (~1.2e-4 per image).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from coverage_layouts import BGEMM_SHAPES, box, kk_of
from gpu_util import assert_parity, check_invariants, image_errors, oracle_channels, run_library

TOL = 1e-3


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def station(n_chan=5, **kw):
    return dataclasses.replace(synth.shrink(synth.workload(2).subs[0], n_chan=n_chan), **kw)


# ------------------------------------------------------------ CPU: plans and refusals
def dry(E, subs, **kw):
    return E.epic_plan(subs, max_time=kw.pop("max_time", 8), flags=E.EPIC_F_DRY_RUN | kw.pop("flags", 0), **kw)


def test_gemm_plans_and_step_sizes(E):
    """Spectra per gridding step: four (dual pol) or eight (single pol) where
    the LDS allows three workgroups per CU; fewer on the 2048-antenna array."""
    cases = [(station(), "fp16", "block", 4), (station(), "fp8", "auto", 4), (station(), "fp16", "dense", 4),
             (synth.workload(1).subs[0], "fp16", "block", 8),
             (synth.workload(5).subs[0], "fp8", "block", 2),
             (synth.workload(5).subs[0], "fp16", "block", 2)]
    for sub, prec, gridder, tb in cases:
        p = dry(E, [sub], precision=prec, gridder=gridder)
        try:
            info = E.epic_plan_query(p)
            assert info["grid_form"][0] == (E.EPIC_GRID_DENSE_GEMM if gridder == "dense" else E.EPIC_GRID_BLOCK_GEMM)
            assert info["grid_step"][0] == tb, (prec, gridder, sub.n_ant)
        finally:
            E.epic_destroy(p)
    p = dry(E, [station()], precision="fp16")
    try:
        assert E.epic_plan_query(p)["grid_form"][0] == E.EPIC_GRID_GATHER
    finally:
        E.epic_destroy(p)


def test_gemm_refusals(E):
    s = station()
    taps = np.random.default_rng(1).standard_normal((5, 256, 2, 3, 3, 2)).astype(np.float32)
    real_xy = taps.copy()
    real_xy[..., 1] = 0.0
    for kw in (dict(precision="fp32", gridder="block"), dict(precision="fp32", gridder="dense"),
               dict(precision="fp8", gridder="gather"),
               dict(precision="fp16", gridder="block", taps=[taps]),            # complex weights
               dict(precision="fp16", gridder="block", taps=[real_xy]),         # X weights != Y weights
               dict(precision="fp8", gridder="block", flags=E.EPIC_F_COMPLEX_WEIGHTS),
               dict(precision="fp16", gridder="block", flags=E.EPIC_F_ONE_LAUNCH)):
        subs = [s, station(n_chan=2)] if kw.get("flags") == E.EPIC_F_ONE_LAUNCH else [s]
        with pytest.raises(E.EpicError) as e:
            dry(E, subs, **kw)
        assert e.value.status == E.EPIC_E_UNSUPPORTED, kw


# ------------------------------------------------------------ GPU parity
@pytest.mark.gpu
@pytest.mark.parametrize("prec,gridder", [("fp16", "block"), ("fp16", "dense"), ("fp8", "block"), ("fp8", "dense")])
def test_station_subset(E, prec, gridder):
    """Station layout, 5 channels, 37 spectra: nine whole steps of four and a
    ragged one, split over several workgroups per channel."""
    sub = station()
    x = synth.samples(sub, 37)
    (gpu,), info = run_library(E, [sub], [x], precision=prec, gridder=gridder)
    assert info["grid_step"][0] == 4
    fro, mx = assert_parity(gpu, oracle.image(sub, x), TOL, f"{prec} {gridder} station subset")
    print(f"{prec} {gridder} station subset: rel err {fro:.2e}, max |d|/peak {mx:.2e}")


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp16", "fp8"])
@pytest.mark.parametrize("cfg,k,nchan,T", [(1, 0, 4, 64), (4, 1, 3, 13), (4, 2, 2, 9), (5, 0, 1, 5)])
def test_other_shapes(E, prec, cfg, k, nchan, T):
    """Single pol 32 x 32 (eight spectra per step), 48 x 48, 96 x 96 and the
    2048-antenna 128 x 128 array (columns over two workgroups)."""
    sub = synth.shrink(synth.workload(cfg).subs[k], n_chan=nchan)
    x = synth.samples(sub, T)
    (gpu,), info = run_library(E, [sub], [x], precision=prec, gridder="block")
    fro, mx = assert_parity(gpu, oracle.image(sub, x), TOL, f"{prec} block cfg{cfg}.{k}")
    print(f"{prec} block cfg{cfg}.{k} (step {info['grid_step'][0]}): rel err {fro:.2e}")


@pytest.mark.gpu
@pytest.mark.parametrize("part", [0, 1])
@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_every_kernel_shape(E, part, prec):
    """Every (N, KK) instantiation of the GEMM-gridding kernel, dual pol, and
    four single-pol ones."""
    shapes = [s for s in BGEMM_SHAPES if (s[0] > 64) == bool(part)]
    subs = [box(N, W, R, P=1 if k % 4 == 3 else 2, seed=300 + 40 * part + k) for k, (N, KK, W, R) in enumerate(shapes)]
    xs = [np.random.default_rng(500 + k).integers(0, 256, (6, 1, s.n_ant, s.n_pol), dtype=np.uint8)
          for k, s in enumerate(subs)]
    gpus, info = run_library(E, subs, xs, precision=prec, gridder="block")
    for k, (s, x, g) in enumerate(zip(subs, xs, gpus)):
        assert kk_of(info["window_max"][k]) == shapes[k][1]
        assert info["grid_form"][k] == E.EPIC_GRID_BLOCK_GEMM
        assert_parity(g, oracle.image(s, x), TOL, f"{prec} block N={s.grid_n} KK={shapes[k][1]} P={s.n_pol}")


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_kernel_size_split_calls_and_determinism(E, prec):
    """K = 5, sigma = 0.8; three calls (13 + 1 + 6 spectra) equal the oracle
    of all 20; a rerun is bit-identical."""
    sub = station(n_chan=3, kernel_k=5)
    x = synth.samples(sub, 20)
    ora = oracle.image(sub, x, kernel_sigma_cells=0.8)
    kw = dict(precision=prec, gridder="block", plan_kw={"kernel_sigma_cells": 0.8})
    (a,), _ = run_library(E, [sub], [x], calls=[13, 1, 6], **kw)
    assert_parity(a, ora, TOL, f"{prec} block K=5 split")
    (b,), _ = run_library(E, [sub], [x], calls=[13, 1, 6], **kw)
    assert np.array_equal(a, b)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_real_gains_rebuild_the_operand(E, prec):
    """Real gains equal for both pols (delay-free amplitude corrections) fold
    into the GEMM operand too: set mid-integration, the image is the sum of
    the two stretches, each with its own weights."""
    import torch
    sub = station(n_chan=2)
    x = synth.samples(sub, 12)
    g = np.ones((2, 256, 2, 2), dtype=np.float32)
    g[..., 1] = 0.0
    amp = np.random.default_rng(3).uniform(0.5, 2.0, (2, 256)).astype(np.float32)
    g[..., 0] = amp[..., None]
    dev = torch.device("cuda", 0)
    plan = E.epic_plan([sub], precision=prec, gridder="block", max_time=12)
    try:
        d = torch.from_numpy(x).to(dev)
        out = torch.empty((2, 4, 64, 64), device=dev)
        E.epic_grid_fft_accumulate(plan, [d[:5]], 5)
        E.epic_set_gains(plan, 0, g)
        E.epic_grid_fft_accumulate(plan, [d[5:]], 7)
        E.epic_readout(plan, [out], 1)
        torch.cuda.synchronize()
        gpu = out.double().cpu().numpy()
    finally:
        E.epic_destroy(plan)
    tp = oracle.taps(sub)                                         # [C][A][P][K][K] complex
    scaled = tp * amp[:, :, None, None, None]
    user = np.stack([scaled.real, scaled.imag], axis=-1).astype(np.float32)
    ora = oracle.image(sub, x[:5]) + oracle.image(sub, x[5:], taps=user)
    assert_parity(gpu, ora, TOL, f"{prec} block gains")


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_full_station_all_channels(E, prec):
    """The station at full size (132 channels, 1000 spectra in one call) with
    block-GEMM gridding, every channel against the oracle; the per-channel
    error is reported."""
    sub, x, ora = oracle_channels(2, 1000)
    (gpu,), _ = run_library(E, [sub], [x], precision=prec, gridder="block")
    fro, mx = image_errors(gpu, ora)
    per_c = fro.max(axis=1)
    print(f"{prec} block station per-channel rel err: max {per_c.max():.2e} (channel {int(per_c.argmax())}), "
          f"median {np.median(per_c):.2e}")
    assert_parity(gpu, ora, TOL, f"{prec} block station, all 132 channels")
    check_invariants(gpu)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_full_large_array_sampled_channels(E, prec):
    """The 2048-antenna array at full size (256 channels, N = 128, 125
    spectra in one call) with block-GEMM gridding, against the oracle on
    three channels; invariants on all."""
    chans = (0, 128, 255)
    sub, x, ora = oracle_channels(5, 125, chans)
    (gpu,), info = run_library(E, [sub], [x], precision=prec, gridder="block")
    for c in chans:
        fro, mx = assert_parity(gpu[c:c + 1], ora[c:c + 1], TOL, f"{prec} block large array channel {c}")
        print(f"{prec} block large array channel {c}: rel err {fro:.2e}, max |d|/peak {mx:.2e}")
    check_invariants(gpu)
