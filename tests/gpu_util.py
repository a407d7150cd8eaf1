"""Helpers of the GPU parity tests: run the library through its C ABI on
seeded inputs and compare with the FP64 oracle per image."""
from __future__ import annotations

import numpy as np

import oracle


def torch_dev():
    import torch
    return torch, torch.device("cuda", 0)


def run_library(E, subs, samples_list, precision="fp32", calls=None, taps=None, nibble_order=0, output=0,
                flags=0, gridder=0, readout_reset=True, plan_kw=None):
    """Plan, accumulate (optionally split into several calls), read out.
    Returns a list of float64 numpy cubes [C][NPP][N][N] and the plan info."""
    torch, dev = torch_dev()
    T = samples_list[0].shape[0]
    calls = calls or [T]
    assert sum(calls) == T
    plan = E.epic_plan(subs, precision=precision, max_time=max(max(calls), 1), taps=taps,
                       nibble_order=nibble_order, output=output, flags=flags, gridder=gridder, **(plan_kw or {}))
    try:
        info = E.epic_plan_query(plan)
        d_samples = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in samples_list]
        outs = [torch.full((s.n_chan, info["npp"][k], s.grid_n, s.grid_n), float("nan"), dtype=torch.float32,
                           device=dev) for k, s in enumerate(subs)]
        t = 0
        for n in calls:
            E.epic_grid_fft_accumulate(plan, [x[t:t + n] for x in d_samples], n)
            t += n
        E.epic_readout(plan, outs, 1 if readout_reset else 0)
        torch.cuda.synchronize()
        res = [o.double().cpu().numpy() for o in outs]
    finally:
        E.epic_destroy(plan)
    return res, info


def image_errors(gpu: np.ndarray, ora: np.ndarray):
    """Per-image relative Frobenius error and max abs error over the channel
    peak.  Cross products (index 2, 3) are normalised by sqrt(|XX| |YY|)."""
    C, npp = ora.shape[:2]
    fro = np.zeros((C, npp))
    mx = np.zeros((C, npp))
    for c in range(C):
        nx = np.linalg.norm(ora[c, 0])
        ny = np.linalg.norm(ora[c, 1]) if npp == 4 else nx
        peak = np.abs(ora[c, : min(npp, 2)]).max()
        for k in range(npp):
            den = np.linalg.norm(ora[c, k]) if k < 2 else np.sqrt(nx * ny)
            fro[c, k] = np.linalg.norm(gpu[c, k] - ora[c, k]) / max(den, 1e-300)
            mx[c, k] = np.abs(gpu[c, k] - ora[c, k]).max() / max(peak, 1e-300)
    return fro, mx


def assert_parity(gpu, ora, tol, what=""):
    assert np.isfinite(gpu).all(), f"{what}: non-finite output"
    fro, mx = image_errors(gpu, ora)
    assert fro.max() <= tol, f"{what}: max per-image relative error {fro.max():.3e} > {tol:.1e}"
    assert mx.max() <= tol, f"{what}: max |diff| / peak {mx.max():.3e} > {tol:.1e}"
    return fro.max(), mx.max()


_ORACLE_CACHE: dict = {}


def oracle_channels(cfg: int, T: int, chans=None) -> tuple:
    """Samples of workload ``cfg`` (T spectra, seeded) and the oracle's image
    cube restricted to ``chans`` (None: every channel, in one threaded oracle
    call), cached per process so that the FP32 and FP16 full-size tests share
    one oracle run."""
    import synth
    key = (cfg, T, None if chans is None else tuple(chans))
    if key not in _ORACLE_CACHE:
        sub = synth.workload(cfg).subs[0]
        x = synth.samples(sub, T)
        if chans is None:
            ora = oracle.image(sub, x)
        else:
            ora = np.zeros((sub.n_chan, 4 if sub.n_pol == 2 else 1, sub.grid_n, sub.grid_n))
            for c in chans:
                ora[c] = oracle.image(sub, x, chans=range(c, c + 1))[c]
        while len(_ORACLE_CACHE) >= 2:   # at most two full-size workloads held at a time
            _ORACLE_CACHE.pop(next(iter(_ORACLE_CACHE)))
        _ORACLE_CACHE[key] = (sub, x, ora)
    return _ORACLE_CACHE[key]


def check_invariants(gpu: np.ndarray):
    """Properties every image cube has: finite, XX (and YY) >= 0, and for
    dual pol |XY*|^2 <= XX * YY per pixel (Cauchy-Schwarz), up to FP32
    rounding."""
    assert np.isfinite(gpu).all()
    if gpu.shape[1] == 1:
        assert (gpu >= 0).all()
        return
    assert (gpu[:, 0] >= 0).all() and (gpu[:, 1] >= 0).all()
    assert (gpu[:, 2] ** 2 + gpu[:, 3] ** 2 <= gpu[:, 0] * gpu[:, 1] * (1 + 1e-4) + 1e-3).all()
