"""Direct imaging on the matrix cores (EPIC_GRID_DIRECT_GEMM) against the FP64
oracle.

Gridding (Eq. 4) and the inverse transform are both linear, so for one
channel their composition is a single matrix: pixel q's field is the sum over
antennas of the antenna's kernel image at q times its field.  The form builds
that matrix once per plan (FP64, split FP16 hi + lo) and forms every pixel's
field as an FP16 product with FP32 accumulation; the products of Eq. 5 and
their sums stay FP32.  No aperture grid and no FFT, so the rounding differs
from the grid-and-FFT forms: the 4-bit fields are exact in FP16, the matrix
carries ~2^-22 relative error, and the FP32 sums over A <= 64 antennas stay
far under the 1e-3 per-image bar of the reduced-precision forms.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from coverage_layouts import box
from gpu_util import assert_parity, check_invariants, oracle_channels, run_library, torch_dev

TOL = 1e-3


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def station64(n_chan=5, **kw):
    """The first 64 antennas of the 256-antenna station, 64 x 64 grid."""
    s = synth.shrink(synth.workload(2).subs[0], n_chan=n_chan, n_ant=64)
    return dataclasses.replace(s, **kw)


def dry(E, subs, **kw):
    return E.epic_plan(subs, max_time=kw.pop("max_time", 8), flags=E.EPIC_F_DRY_RUN | kw.pop("flags", 0), **kw)


# ------------------------------------------------------------ CPU: plans and refusals
def test_direct_plans(E):
    """The form is taken on request for arrays of at most 64 antennas on
    grids up to 64; a step holds 16 single-pol or 8 dual-pol spectra."""
    for sub, step in ((synth.workload(1).subs[0], 16), (station64(), 8), (box(48, 20, 18, P=2, n_extra=40), 8)):
        p = dry(E, [sub], precision="fp16", gridder="direct")
        try:
            info = E.epic_plan_query(p)
            assert info["grid_form"][0] == E.EPIC_GRID_DIRECT_GEMM
            assert info["grid_step"][0] == step
        finally:
            E.epic_destroy(p)


def test_direct_refusals(E):
    s = station64()
    rng = np.random.default_rng(1)
    cplx = rng.standard_normal((5, 64, 2, 3, 3, 2)).astype(np.float32)
    real_xy = cplx.copy()
    real_xy[..., 1] = 0.0                                   # real, but X != Y
    wide = synth.shrink(synth.workload(6).subs[0], n_chan=2, n_ant=64)      # N = 256
    for subs, kw in (([s], dict(precision="fp32")), ([s], dict(precision="fp8")),
                     ([synth.shrink(synth.workload(2).subs[0], n_chan=2)], dict(precision="fp16")),   # 256 antennas
                     ([wide], dict(precision="fp16")),
                     ([s], dict(precision="fp16", taps=[cplx])),
                     ([s], dict(precision="fp16", taps=[real_xy])),
                     ([s, station64(n_chan=2)], dict(precision="fp16", flags=E.EPIC_F_ONE_LAUNCH))):
        with pytest.raises(E.EpicError) as e:
            dry(E, subs, gridder="direct", **kw)
        assert e.value.status == E.EPIC_E_UNSUPPORTED, (kw, [x.n_ant for x in subs])


# ------------------------------------------------------------ GPU parity
@pytest.mark.gpu
def test_small_array_every_channel(E):
    """The 16-antenna single-pol array (32 x 32, four channels) with 1000
    spectra in one call, every channel against the oracle."""
    sub, x, ora = oracle_channels(1, 1000)
    (gpu,), info = run_library(E, [sub], [x], precision="fp16", gridder="direct")
    assert info["grid_form"][0] == E.EPIC_GRID_DIRECT_GEMM
    fro, mx = assert_parity(gpu, ora, TOL, "direct, 16-antenna array")
    print(f"direct 16-antenna array: rel err {fro:.2e}, max |d|/peak {mx:.2e}")
    check_invariants(gpu)


@pytest.mark.gpu
def test_station64_dual_pol(E):
    """64 antennas, dual pol, 64 x 64, 37 spectra: four 16-antenna blocks,
    four whole steps of eight spectra and a ragged one per time chunk."""
    sub = station64()
    x = synth.samples(sub, 37)
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16", gridder="direct")
    fro, mx = assert_parity(gpu, oracle.image(sub, x), TOL, "direct, 64-antenna station")
    print(f"direct 64-antenna station: rel err {fro:.2e}, max |d|/peak {mx:.2e}")


@pytest.mark.gpu
@pytest.mark.parametrize("N,W,R,A,P", [(32, 13, 9, 7, 2), (32, 20, 29, 20, 1), (48, 25, 31, 33, 2),
                                        (48, 16, 12, 48, 1), (64, 30, 18, 17, 2), (64, 61, 50, 64, 1)])
def test_every_block_count(E, N, W, R, A, P):
    """One, two, three and four 16-antenna blocks (ragged last block), both
    pol counts, every grid size the form takes."""
    sub = box(N, W, R, P=P, n_extra=A - 2, seed=N + A)
    x = np.random.default_rng(A).integers(0, 256, (11, 1, A, P), dtype=np.uint8)
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16", gridder="direct")
    assert_parity(gpu, oracle.image(sub, x), TOL, f"direct N={N} A={A} P={P}")


@pytest.mark.gpu
def test_kernel_size_split_calls_and_determinism(E):
    """K = 5, sigma = 0.8, 48 antennas; three calls (13 + 1 + 6 spectra)
    equal the oracle of all 20; a rerun is bit-identical."""
    sub = station64(n_chan=3, kernel_k=5)
    sub = synth.shrink(sub, n_ant=48)
    x = synth.samples(sub, 20)
    ora = oracle.image(sub, x, kernel_sigma_cells=0.8)
    kw = dict(precision="fp16", gridder="direct", plan_kw={"kernel_sigma_cells": 0.8})
    (a,), _ = run_library(E, [sub], [x], calls=[13, 1, 6], **kw)
    assert_parity(a, ora, TOL, "direct K=5 split")
    (b,), _ = run_library(E, [sub], [x], calls=[13, 1, 6], **kw)
    assert np.array_equal(a, b)


@pytest.mark.gpu
def test_complex_user_taps_single_pol(E):
    """Complex taps (a single-pol array takes any weights): the kernel image
    is complex and the matrix's real form carries both parts."""
    sub = synth.workload(1).subs[0]
    tp = np.random.default_rng(7).standard_normal((4, 16, 1, 3, 3, 2)).astype(np.float32)
    x = synth.samples(sub, 24)
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16", gridder="direct", taps=[tp],
                            flags=E.EPIC_F_COMPLEX_WEIGHTS)
    assert_parity(gpu, oracle.image(sub, x, taps=tp), TOL, "direct complex taps")


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["single-pol complex", "dual-pol real"])
def test_gains_rebuild_the_matrix(E, which):
    """Gains set mid-integration rebuild the matrix: the image is the sum of
    the two stretches, each with its own weights."""
    torch, dev = torch_dev()
    rng = np.random.default_rng(3)
    if which == "single-pol complex":
        sub = synth.workload(1).subs[0]
        g = rng.uniform(-1.5, 1.5, (4, 16, 1, 2)).astype(np.float32)
        gc = g[..., 0] + 1j * g[..., 1]                              # [C][A][P]
    else:
        sub = station64(n_chan=2)
        amp = rng.uniform(0.5, 2.0, (2, 64)).astype(np.float32)
        g = np.zeros((2, 64, 2, 2), dtype=np.float32)
        g[..., 0] = amp[..., None]
        gc = g[..., 0].astype(np.complex128)
    x = synth.samples(sub, 12)
    npp = 4 if sub.n_pol == 2 else 1
    flags = E.EPIC_F_COMPLEX_WEIGHTS if sub.n_pol == 1 else 0      # phase gains need complex weights
    plan = E.epic_plan([sub], precision="fp16", gridder="direct", max_time=12, flags=flags)
    try:
        d = torch.from_numpy(x).to(dev)
        out = torch.empty((sub.n_chan, npp, sub.grid_n, sub.grid_n), device=dev)
        E.epic_grid_fft_accumulate(plan, [d[:5]], 5)
        E.epic_set_gains(plan, 0, g)
        E.epic_grid_fft_accumulate(plan, [d[5:]], 7)
        E.epic_readout(plan, [out], 1)
        torch.cuda.synchronize()
        gpu = out.double().cpu().numpy()
    finally:
        E.epic_destroy(plan)
    tp = oracle.taps(sub)                                           # [C][A][P][K][K] complex
    scaled = tp * gc[:, :, :, None, None]
    user = np.stack([scaled.real, scaled.imag], axis=-1).astype(np.float32)
    ora = oracle.image(sub, x[:5]) + oracle.image(sub, x[5:], taps=user)
    assert_parity(gpu, ora, TOL, f"direct gains ({which})")


@pytest.mark.gpu
def test_noalloc_entry_point(E):
    """The allocation-free entry point runs the direct form too: two calls,
    the second smaller, against accumulate + read-out of the same plan."""
    torch, dev = torch_dev()
    sub = station64(n_chan=3)
    x = torch.from_numpy(synth.samples(sub, 40)).to(dev)
    plan = E.epic_plan([sub], precision="fp16", gridder="direct", max_time=40)
    try:
        for n in (40, 9):
            a = torch.full((3, 4, 64, 64), float("nan"), device=dev)
            b = torch.full((3, 4, 64, 64), float("nan"), device=dev)
            E.epic_image_noalloc(plan, [x[:n]], n, [a])
            E.epic_grid_fft_accumulate(plan, [x[:n]], n)
            E.epic_readout(plan, [b], 1)
            torch.cuda.synchronize()
            assert_parity(a.double().cpu().numpy(), b.double().cpu().numpy(), 1e-5, f"direct noalloc {n}")
    finally:
        E.epic_destroy(plan)


@pytest.mark.gpu
def test_autotuner_times_the_direct_form(E):
    """With the library's choice of gridder and EPIC_F_AUTOTUNE, the small
    array's plan times the direct form beside the gather and block-GEMM forms;
    whichever wins, the image matches the oracle."""
    sub = synth.workload(1).subs[0]
    x = synth.samples(sub, 64)
    (gpu,), info = run_library(E, [sub], [x], precision="fp16", flags=E.EPIC_F_AUTOTUNE)
    assert info["autotuned"] == 1
    print(f"autotuned 16-antenna array: grid form {info['grid_form'][0]}")
    assert_parity(gpu, oracle.image(sub, x), TOL, "autotuned small array")
