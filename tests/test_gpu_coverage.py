"""Parity at every compiled variant of the hot kernels and at every kernel
size and width the ABI accepts.

* FP32: every fixed-length row fold (two or three blocks of 8, last-block
  tails 1, 2, 4, 8) and every branch of the generic fold (one block; two;
  three or more, which runs the middle-block loop; each tail), at N = 32, 64
  and, for the generic fold without LDS twiddles, N = 96.
* FP16: every (N, KK) instantiation of the matrix-core kernel, every shape of
  the single persistent launch, and the weight modes (one real weight shared
  by both pols, real per pol, complex; single and dual pol).
* Gaussian kernels of K = 1, 5, 7 taps and sigma 0.35 and 0.8 cells in both
  forms (Eq. 4's W_a; Sec. 3.1 grids each antenna through its kernel).

The CPU tests check, through dry-run plans and the library's own geometry,
that the layouts reach every class the kernels dispatch on; the GPU tests
compare each layout's image with the FP64 oracle.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from coverage_layouts import (ALL_FIXED, ALL_GENERIC, BATCH_SHAPES, FOLD_WINDOWS, MFMA_SHAPES, box, fold_class,
                              kk_of, windows_of)
from gpu_util import assert_parity, run_library

TOL32, TOL16 = 1e-5, 1e-3


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def fold_subs(N):
    subs = [box(N, W, R, P=2 if k % 4 else 1, seed=100 * N + k) for k, (W, R) in enumerate(FOLD_WINDOWS)]
    return subs


def mfma_subs(shapes, P=2, seed=0):
    return [box(N, W, R, P=P, seed=seed + k) for k, (N, KK, W, R) in enumerate(shapes)]


def samples_for(sub, T, seed):
    return np.random.default_rng(seed).integers(0, 256, (T, sub.n_chan, sub.n_ant, sub.n_pol), dtype=np.uint8)


# ------------------------------------------------------------ CPU: the layouts reach every class
@pytest.mark.parametrize("N", [32, 64, 96])
def test_fold_layouts_reach_every_fold(E, N):
    plan = E.epic_plan(fold_subs(N), max_time=4, flags=E.EPIC_F_DRY_RUN)
    try:
        rows, cols = set(), set()
        for k, (W, R) in enumerate(FOLD_WINDOWS):
            w, r = windows_of(E.epic_debug_geometry(plan, k), 3)
            assert (int(w[0]), int(r[0])) == (W, R)
            rows.add(fold_class(W, fixed=N <= 64))
            cols.add(fold_class(R, fixed=False))
    finally:
        E.epic_destroy(plan)
    assert cols == ALL_GENERIC
    if N <= 64:
        assert ALL_FIXED <= rows and {("generic", 1, 0), ("generic", 3, 1), ("generic", 3, 2),
                                      ("generic", 3, 4), ("generic", 3, 8)} <= rows
    else:
        assert rows == ALL_GENERIC


def test_mfma_layouts_reach_every_shape(E):
    got = set()
    for part in (0, 1):   # at most 16 sub-arrays per plan
        subs = mfma_subs([s for s in MFMA_SHAPES if (s[0] > 64) == bool(part)])
        plan = E.epic_plan(subs, precision="fp16", max_time=4, flags=E.EPIC_F_DRY_RUN)
        try:
            info = E.epic_plan_query(plan)
            got |= {(s.grid_n, kk_of(info["window_max"][k])) for k, s in enumerate(subs)}
        finally:
            E.epic_destroy(plan)
    assert got == {(N, KK) for N, KK, _, _ in MFMA_SHAPES}
    assert len(got) == 25


def test_batch_layouts_reach_every_shape(E):
    subs = mfma_subs(BATCH_SHAPES)
    plan = E.epic_plan(subs, precision="fp16", max_time=4, flags=E.EPIC_F_DRY_RUN | E.EPIC_F_ONE_LAUNCH)
    try:
        info = E.epic_plan_query(plan)
        assert info["batched"] == 1
        got = {(s.grid_n, kk_of(info["window_max"][k])) for k, s in enumerate(subs)}
    finally:
        E.epic_destroy(plan)
    assert got == {(N, KK) for N, KK, _, _ in BATCH_SHAPES} and len(got) == 13


# ------------------------------------------------------------ GPU parity
@pytest.mark.gpu
@pytest.mark.parametrize("N", [32, 64, 96])
def test_fp32_every_fold(E, N):
    """Thirteen single-channel arrays (dual and single pol) whose windows
    reach every row and column fold of the FP32 kernel at this grid size."""
    subs = fold_subs(N)
    xs = [samples_for(s, 3, 7 + k) for k, s in enumerate(subs)]
    gpus, _ = run_library(E, subs, xs)
    for k, (s, x, g) in enumerate(zip(subs, xs, gpus)):
        assert_parity(g, oracle.image(s, x), TOL32, f"N={N} window {s.W}x{s.R} P={s.n_pol}")


@pytest.mark.gpu
@pytest.mark.parametrize("part", [0, 1])
def test_fp16_every_mfma_shape(E, part):
    """Every (N, KK) matrix-core kernel (N = 32 .. 256), one single-channel
    array each; the N <= 64 half also runs the real-per-pol and complex
    weight modes and a single-pol array."""
    shapes = [s for s in MFMA_SHAPES if (s[0] > 64) == bool(part)]
    subs = mfma_subs(shapes, seed=40 * part)
    taps = [None] * len(subs)
    if part == 0:
        rng = np.random.default_rng(5)
        subs[1] = dataclasses.replace(subs[1], n_pol=1)                      # P = 1, real weights
        t = rng.standard_normal((1, subs[3].n_ant, 2, 3, 3, 2)).astype(np.float32)
        t[..., 1] = 0.0                                                      # real, X != Y
        taps[3] = t
        subs[4] = dataclasses.replace(subs[4], n_pol=1)
        taps[4] = rng.standard_normal((1, subs[4].n_ant, 1, 3, 3, 2)).astype(np.float32)   # P = 1 complex
        taps[6] = rng.standard_normal((1, subs[6].n_ant, 2, 3, 3, 2)).astype(np.float32)   # P = 2 complex
    xs = [samples_for(s, 4, 11 + k) for k, s in enumerate(subs)]
    gpus, info = run_library(E, subs, xs, precision="fp16", taps=taps)
    for k, (s, x, g) in enumerate(zip(subs, xs, gpus)):
        assert kk_of(info["window_max"][k]) == shapes[k][1]
        assert_parity(g, oracle.image(s, x, taps=taps[k]), TOL16, f"fp16 N={s.grid_n} KK={shapes[k][1]}")


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["shared", "complex", "real", "single", "single-complex"])
def test_batch_every_shape_one_launch(E, mode):
    """All thirteen shapes of the single persistent launch in one launch
    (dual pol, one real weight shared by both pols); then a third of them
    with complex weights, with real per-pol weights, single-pol, and
    single-pol complex."""
    subs = mfma_subs(BATCH_SHAPES, seed=70)
    flags = E.EPIC_F_ONE_LAUNCH
    taps = None
    if mode == "complex":
        flags |= E.EPIC_F_COMPLEX_WEIGHTS
        subs = subs[::3]
    if mode == "real":
        subs = subs[2::3]
        rng = np.random.default_rng(6)
        taps = []
        for s in subs:
            t = rng.standard_normal((1, s.n_ant, 2, 3, 3, 2)).astype(np.float32)
            t[..., 1] = 0.0
            taps.append(t)
    if mode.startswith("single"):
        subs = [dataclasses.replace(s, n_pol=1) for s in subs[1::3]]
        if mode == "single-complex":
            flags |= E.EPIC_F_COMPLEX_WEIGHTS
    xs = [samples_for(s, 5, 90 + k) for k, s in enumerate(subs)]
    gpus, info = run_library(E, subs, xs, precision="fp16", flags=flags, taps=taps)
    assert info["batched"] == 1
    for k, (s, x, g) in enumerate(zip(subs, xs, gpus)):
        assert_parity(g, oracle.image(s, x, taps=None if taps is None else taps[k]), TOL16,
                      f"batch {mode} N={s.grid_n} window {s.W}x{s.R}")


def station(n_chan=3, k=3):
    return dataclasses.replace(synth.shrink(synth.workload(2).subs[0], n_chan=n_chan), kernel_k=k)


@pytest.mark.gpu
@pytest.mark.parametrize("k,sigma", [(1, 0.5), (5, 0.8), (5, 0.35), (7, 0.8)])
def test_fp32_kernel_sizes_and_widths(E, k, sigma):
    """Gaussian kernels of K = 1, 5, 7 taps and sigma != 0.5 (station layout,
    3 channels, 12 spectra) in the FP32 form."""
    sub = station(k=k)
    x = synth.samples(sub, 12)
    (gpu,), _ = run_library(E, [sub], [x], plan_kw={"kernel_sigma_cells": sigma})
    fro, mx = assert_parity(gpu, oracle.image(sub, x, kernel_sigma_cells=sigma), TOL32, f"fp32 K={k} s={sigma}")
    print(f"fp32 K={k} sigma={sigma}: rel err {fro:.2e}")


@pytest.mark.gpu
@pytest.mark.parametrize("k,sigma", [(1, 0.5), (5, 0.8), (7, 0.35)])
def test_fp16_kernel_sizes_and_widths(E, k, sigma):
    """The same in the FP16 matrix-core form."""
    sub = station(k=k)
    x = synth.samples(sub, 12)
    (gpu,), _ = run_library(E, [sub], [x], precision="fp16", plan_kw={"kernel_sigma_cells": sigma})
    fro, mx = assert_parity(gpu, oracle.image(sub, x, kernel_sigma_cells=sigma), TOL16, f"fp16 K={k} s={sigma}")
    print(f"fp16 K={k} sigma={sigma}: rel err {fro:.2e}")


@pytest.mark.gpu
def test_batched_kernel_size_five(E):
    """K = 5, sigma = 0.8 in the single persistent launch of two sub-arrays."""
    s1 = dataclasses.replace(synth.shrink(synth.workload(4).subs[0], n_chan=2), kernel_k=5)
    s2 = dataclasses.replace(synth.shrink(synth.workload(4).subs[1], n_chan=3), kernel_k=5)
    xs = [synth.samples(s1, 6), synth.samples(s2, 6)]
    gpus, info = run_library(E, [s1, s2], xs, precision="fp16", flags=E.EPIC_F_ONE_LAUNCH,
                             plan_kw={"kernel_sigma_cells": 0.8})
    assert info["batched"] == 1
    for s, x, g in zip((s1, s2), xs, gpus):
        assert_parity(g, oracle.image(s, x, kernel_sigma_cells=0.8), TOL16, f"batch K=5 N={s.grid_n}")
