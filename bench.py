#!/usr/bin/env python3
"""Benchmark of the EPIC/MOFF imaging hot path on one MI355X.

A step is one pass of the whole path over one batch: epic_grid_fft_accumulate
over the workload's spectra (unpack, grid, 2D transform, polarisation products,
accumulate) followed by one epic_readout (ordered reduce + reset).  Inputs are
resident in HBM before the timed region.  Prints ONE JSON line.

Workload (default): the station-scale FP32 configuration -- 256 dual-pol
antennas in a 100 m x 110 m ellipse, 132 channels of 25 kHz from 40 MHz, 64x64
grid at 1 wavelength, 3x3 kernels, 1000 spectra (40 ms) per step, seeded
synthetic 4+4-bit samples (noise + 3 point sources).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector, published (packed issue)
FP32_NONPACKED_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP16_MFMA_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0


def algorithmic_flops_per_ct(sub) -> float:
    """Nominal flops of one (channel, spectrum): complex gridding 8 per tap per
    pol, a 2D FFT of 10 N^2 log2 N per pol (5 n log2 n per 1-D transform), and
    the products (16 per pixel dual pol, 4 single)."""
    A, P, N, K = sub.n_ant, sub.n_pol, sub.grid_n, sub.kernel_k
    grid = P * A * K * K * 8
    fft = P * 10 * N * N * math.log2(N)
    prod = (16 if P == 2 else 4) * N * N
    return grid + fft + prod


# Sources of each precision's hot kernel: the counter-based traffic in
# profiles/traffic.json is reported only while their hash still matches.
KERNEL_SOURCES = {
    "fp32": ["kernels_fp32.hip", "epic_device.hpp", "epic_gather.hpp", "epic_sched.hpp", "epic_internal.hpp"],
    "fp16": ["kernels_mfma.hip", "epic_device.hpp", "epic_gather.hpp", "epic_sched.hpp", "epic_internal.hpp"],
}


def sources_sha256(precision):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(precision, []):
        with open(os.path.join(ROOT, "paper_2301_09662_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def counter_traffic(precision, workload):
    """HBM bytes per launch of the hot kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter runs (scaled by the plain-copy calibration), or None
    when there are none for this workload or the kernel changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        entry = json.load(fh).get("kernels", {}).get(f"{precision}:{workload}")
    if not entry or entry.get("sources_sha256") != sources_sha256(precision):
        return None
    return entry["bytes_per_launch"]


MFMA_FLOPS = 2 * 16 * 16 * 32     # one v_mfma_f32_16x16x32_f16


def mfma_ops_per_spectrum(plan, subs):
    """MFMA 16x16x32 instructions the matrix-core kernel executes for one
    spectrum of every channel of every sub-array, from the plan's shapes: per
    column part, the row pass takes ceil(M1/16) x (2 NK/16) x KK products
    (M1 = P x window rows rounded up to 4) and the column pass
    (N/16) x (NK/16) x P x 2 x KK, with KK 32-deep steps covering the largest
    window extent (rounded up to 8) and NK = N/KS columns per part."""
    from paper_2301_09662_amd import epic as E
    total = 0
    for k, s in enumerate(subs):
        g = E.epic_debug_geometry(plan, k)                     # [C][A][(x, y)] nearest cells
        hk = s.kernel_k // 2
        R = g[:, :, 1].max(1) - g[:, :, 1].min(1) + 1 + 2 * hk
        W = g[:, :, 0].max(1) - g[:, :, 0].min(1) + 1 + 2 * hk
        ext = max(-(-int(R.max()) // 8) * 8, -(-int(W.max()) // 8) * 8)
        KK = -(-ext // 16)
        N, P = s.grid_n, s.n_pol
        KS = 2 if N > 64 else 1
        NK = N // KS
        M1 = P * ((R + 3) // 4 * 4)
        per_c = KS * (-(-M1 // 16) * (2 * NK // 16) * KK + (N // 16) * (NK // 16) * P * 2 * KK)
        total += int(per_c.sum())
    return total


def mfma_fraction(info, kern_ms):
    """Executed FP16 MFMA rate of a matrix-core call against the dense peak."""
    ops = info["mfma_ops_per_call"]
    tflops = ops * MFMA_FLOPS / (kern_ms * 1e-3) / 1e12
    return {"executed_ops_per_call": ops, "executed_tflops": tflops, "peak": FP16_MFMA_PEAK_TFLOPS,
            "frac": tflops / FP16_MFMA_PEAK_TFLOPS, "source": "tile counts of the plan's shapes"}


def rel_image_errors(img, ref):
    """Per-image relative Frobenius error [C][NPP] of img against ref; the
    cross products are normalised by sqrt(|XX| |YY|) of ref."""
    C, npp = ref.shape[:2]
    out = np.zeros((C, npp))
    for c in range(C):
        nx = np.linalg.norm(ref[c, 0])
        ny = np.linalg.norm(ref[c, 1]) if npp == 4 else nx
        for k in range(npp):
            den = np.linalg.norm(ref[c, k]) if k < 2 else np.sqrt(nx * ny)
            out[c, k] = np.linalg.norm(img[c, k] - ref[c, k]) / max(den, 1e-300)
    return out


def cpu_baseline(sub, samples, budget_s=15.0):
    """Time the FP64 oracle on a bounded sample of the same workload: all
    channels over the first T_s spectra, T_s sized for ~budget_s of wall time."""
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    probe_t = 4
    t0 = time.perf_counter()
    oracle.image(sub, samples[:probe_t], n_threads=cores)
    dt = time.perf_counter() - t0
    T_s = int(max(probe_t, min(samples.shape[0], budget_s / max(dt, 1e-6) * probe_t)))
    t0 = time.perf_counter()
    oracle.image(sub, samples[:T_s], n_threads=cores)
    wall = time.perf_counter() - t0
    n = sub.n_ant * sub.n_pol * sub.n_chan * T_s
    return {"value": n / wall, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"all {sub.n_chan} channels x first {T_s} of {samples.shape[0]} spectra "
                      f"({wall:.1f} s wall, FP64 C loops, OpenMP over channels)"}


def numpy_fft_image(sub, x, c):
    """One channel's image cube [NPP][N][N] computed the plain vectorised way
    in FP32 NumPy/SciPy: nearest-cell Gaussian gridding as a sparse matrix
    (taps times the (-1)^(x+y) centring), unnormalised exp(+2 pi i) 2D FFT,
    products XX*, YY*, Re XY*, Im XY* summed over the spectra of x
    (uint8 [T][A][P], nibble order 0).  CPU context for the benchmark, not an
    oracle."""
    import scipy.sparse as sp
    N, K, P, A = sub.grid_n, sub.kernel_k, sub.n_pol, sub.n_ant
    hk = K // 2
    b = np.arange(256)
    hi, lo = ((b >> 4) ^ 8) - 8, ((b & 15) ^ 8) - 8
    lut = (hi + 1j * lo).astype(np.complex64)
    lam = 299792458.0 / (sub.freq0_hz + c * sub.dfreq_hz)
    g = sub.ant_xy / lam / sub.grid_dl + N / 2                       # [A][(x, y)] in cells
    p0 = np.floor(g + 0.5).astype(np.int64)
    d = np.arange(-hk, hk + 1)
    cx = p0[:, 0, None, None] + d[None, None, :]                      # [A][dy][dx]
    cy = p0[:, 1, None, None] + d[None, :, None]
    w = np.exp(-((cx - g[:, 0, None, None]) ** 2 + (cy - g[:, 1, None, None]) ** 2) / (2 * 0.5 ** 2))
    w /= w.sum(axis=(1, 2), keepdims=True)
    w *= np.where((cx + cy) % 2 == 0, 1.0, -1.0)
    M = sp.csr_matrix((w.ravel().astype(np.float32), ((cy * N + cx).ravel(), np.repeat(np.arange(A), K * K))),
                      shape=(N * N, A))
    T = x.shape[0]
    E = lut[x]                                                        # [T][A][P]
    G = (M @ E.transpose(1, 0, 2).reshape(A, T * P)).reshape(N, N, T, P)
    F = np.fft.ifft2(G, axes=(0, 1)).astype(np.complex64) * np.float32(N * N)
    X = F[..., 0]
    out = [np.sum(np.abs(X) ** 2, axis=2)]
    if P == 2:
        Y = F[..., 1]
        xy = np.sum(X * np.conj(Y), axis=2)
        out += [np.sum(np.abs(Y) ** 2, axis=2), xy.real, xy.imag]
    return np.stack(out)


def cpu_numpy_fft(sub, samples, budget_s=10.0):
    """Time numpy_fft_image on the first channels of the workload (all
    spectra), as many as fit ~budget_s; NumPy's FFT and SciPy's sparse
    product run on one thread."""
    C = sub.n_chan
    numpy_fft_image(sub, samples[:2, 0], 0)   # imports and first-call set-up, untimed
    t0 = time.perf_counter()
    numpy_fft_image(sub, samples[:, 0], 0)
    dt = time.perf_counter() - t0
    n_c = int(max(1, min(C, budget_s / max(dt, 1e-6))))
    t0 = time.perf_counter()
    for c in range(n_c):
        numpy_fft_image(sub, samples[:, c], c)
    wall = time.perf_counter() - t0
    n = sub.n_ant * sub.n_pol * n_c * samples.shape[0]
    return {"value": n / wall, "unit": "samples/s", "cores": 1, "kind": "numpy-fft (context, not an oracle)",
            "sample": f"first {n_c} of {C} channels x all {samples.shape[0]} spectra ({wall:.1f} s wall, "
                      f"FP32 sparse gridding + FFT)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cfg", type=int, default=2, help="workload config (default: station FP32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reduced", action="store_true", help="skip the FP16 matrix-core leg")
    ap.add_argument("--precision", choices=["fp32", "fp16", "fp8"], default=None,
                    help="override the workload's own precision")
    ap.add_argument("--no-graph", action="store_true", help="batched workloads: eager launches instead of graph replay")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times) and exit: the reference for "
                         "scaling the FETCH_SIZE / WRITE_SIZE hardware counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "repeats": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(channels shard across GPUs with no exchange; not built here)"}))
        sys.exit(2)

    import torch
    from paper_2301_09662_amd import epic as E

    wl = synth.workload(args.cfg)
    subs = wl.subs
    T = wl.n_time
    dev = torch.device("cuda", 0)
    host = [synth.samples(s, T) for s in subs]
    d_samples = [torch.from_numpy(x).to(dev) for x in host]
    stream = torch.cuda.current_stream()
    samples_per_step = sum(s.n_ant * s.n_pol * s.n_chan * T for s in subs)
    flops_per_launch = sum(algorithmic_flops_per_ct(s) * s.n_chan * T for s in subs)

    def run(precision, steps, warmup, flags=0):
        plan = E.epic_plan(subs, precision=precision, max_time=T, flags=flags)
        info = E.epic_plan_query(plan)
        outs = [torch.empty((s.n_chan, info["npp"][k], s.grid_n, s.grid_n), dtype=torch.float32, device=dev)
                for k, s in enumerate(subs)]

        def step(ev=None):
            if ev is not None:
                ev[0].record(stream)
            E.epic_grid_fft_accumulate(plan, d_samples, T, stream)
            if ev is not None:
                ev[1].record(stream)
            E.epic_readout(plan, outs, 1, stream)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        if precision == "fp16":
            info = dict(info, mfma_ops_per_call=mfma_ops_per_spectrum(plan, subs) * T)
        E.epic_destroy(plan)
        return wall / steps * 1e3, kern_ms, [o.double().cpu().numpy() for o in outs], info

    # each workload's own precision; the uneven batch of sub-arrays runs as
    # one autotuned persistent launch replayed from a hipGraph
    # the large array's FP8 form is not built: its reduced-precision leg is FP16
    precision = args.precision or ("fp16" if wl.precision == "fp8" else wl.precision)
    flags = 0
    if len(subs) > 1:
        flags = E.EPIC_F_AUTOTUNE | (0 if args.no_graph else E.EPIC_F_GRAPH)
    ms_per_step, kern_ms, img32, info32 = run(precision, args.steps, args.warmup, flags)
    achieved = flops_per_launch / (kern_ms * 1e-3) / 1e12
    res = {
        "metric": "imaged E-field samples/s (ant*chan*pol*t)",
        "value": samples_per_step / (ms_per_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precision == "fp32" else "f16 operands, f32 accumulate",
        "data": "synthetic (seeded 4+4-bit noise + point sources, LWA-station shapes)",
        "config": {"workload": f"{wl.name}: " + "; ".join(
            f"{s.n_ant} ant x {s.n_pol} pol, {s.n_chan} ch, N={s.grid_n}, dl={s.grid_dl}" for s in subs)
            + f", T={T} spectra per step", "n_time": T, "precision": precision,
            "plan": {k: info32[k] for k in ("batched", "can_batch", "form_ms", "autotuned", "graph", "weight",
                                            "slots", "lds_bytes")}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": counter_traffic(precision, wl.name),
                     "kernel_ms": kern_ms, "algorithmic_flops_per_launch": flops_per_launch,
                     "frac_of_nonpacked_issue": achieved / FP32_NONPACKED_TFLOPS},
    }
    if res["roofline"]["traffic"] is not None:
        res["roofline"]["hbm_frac"] = res["roofline"]["traffic"] / (kern_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
    if precision == "fp16":
        # matrix-core form: the kernel is issue bound on its vector work
        # (gathering, FP16 packing, products); executed MFMA work for context
        res["roofline"]["mfma"] = mfma_fraction(info32, kern_ms)
    red_form = not args.no_reduced and precision == "fp32"
    if red_form:
        try:
            ms16, kern16, img16, info16 = run("fp16", args.steps, args.warmup)
        except E.EpicError as err:   # no matrix-core kernel for this grid size
            res["reduced_precision"] = {"precision": "fp16", "unavailable": str(err)}
            red_form = False
    if red_form:
        # error of the FP16 form per image against the FP32 result (all channels);
        # its parity with the FP64 oracle is the tests' business
        errs = [rel_image_errors(a, b).max() for a, b in zip(img16, img32)]
        red = {"precision": "fp16", "value": samples_per_step / (ms16 * 1e-3), "ms_per_step": ms16,
               "kernel_ms": kern16, "speedup_vs_fp32": ms_per_step / ms16,
               "max_rel_image_err_vs_fp32_all_channels": float(max(errs)),
               "achieved_algorithmic_tflops": flops_per_launch / (kern16 * 1e-3) / 1e12,
               "mfma": mfma_fraction(info16, kern16)}
        res["reduced_precision"] = red
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(subs[0], host[0])
        res["cpu_numpy_fft"] = cpu_numpy_fft(subs[0], host[0])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
