#!/usr/bin/env python3
"""Benchmark of the EPIC/MOFF imaging hot path on one MI355X.

A step is one pass of the whole path over one batch: epic_grid_fft_accumulate
over the workload's spectra (unpack, grid, 2D transform, polarisation products,
accumulate) followed by one epic_readout (ordered reduce + reset).  Inputs are
resident in HBM before the timed region.  Prints ONE JSON line.

Besides the workload's own form, the reduced-precision legs time the same
shape with the transforms on the FP16 matrix cores and gridding either as the
FP32 gather or as a product on the matrix cores (block-sparse FP16 and FP8
operands, and the dense kernel matrix in FP16).  The FP64 oracle, timed on the host's cores, also gives every form's
per-channel image error over the same spectra.

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
FP16_MFMA_PEAK_TFLOPS = 2500.0
FP8_MFMA_PEAK_TFLOPS = 5000.0
HBM_PEAK_GBS = 8000.0
TOL = {"fp32": 1e-5, "fp16": 1e-3, "fp8": 1e-3}


def algorithmic_flops_per_ct(sub) -> float:
    """Nominal flops of one (channel, spectrum): complex gridding 8 per tap per
    pol, a 2D FFT of 10 N^2 log2 N per pol (5 n log2 n per 1-D transform), and
    the products (16 per pixel dual pol, 4 single)."""
    A, P, N, K = sub.n_ant, sub.n_pol, sub.grid_n, sub.kernel_k
    grid = P * A * K * K * 8
    fft = P * 10 * N * N * math.log2(N)
    prod = (16 if P == 2 else 4) * N * N
    return grid + fft + prod


# Sources of each hot-kernel family: the counter-based figures in
# profiles/traffic.json and profiles/valu.json are reported only while their
# hash still matches.
KERNEL_SOURCES = {
    "fp32": ["kernels_fp32.hip", "epic_device.hpp", "epic_gather.hpp", "epic_sched.hpp", "epic_internal.hpp"],
    "fp16": ["kernels_mfma.hip", "epic_mfma.hpp", "epic_device.hpp", "epic_gather.hpp", "epic_sched.hpp",
             "epic_internal.hpp"],
    "bgemm": ["kernels_bgemm.hip", "epic_mfma.hpp", "epic_device.hpp", "epic_sched.hpp", "epic_internal.hpp"],
    "dense": ["kernels_bgemm.hip", "epic_mfma.hpp", "epic_device.hpp", "epic_sched.hpp", "epic_internal.hpp"],
    "direct": ["kernels_direct.hip", "epic_mfma.hpp", "epic_device.hpp", "epic_gather.hpp", "epic_internal.hpp"],
}


def kernel_family(precision, info, k=0):
    """Hot kernel of a plan's sub-array k: the FP32 kernel, the matrix-core
    gather kernel, the GEMM-gridding kernel (FP16 / FP8; dense or block-sparse
    tables, counted apart) or the direct form."""
    if precision == "fp32":
        return "fp32"
    return {1: "fp16", 2: "dense", 3: "bgemm", 4: "direct"}[info["grid_form"][k]]


def sources_sha256(family):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_2301_09662_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def counter_entry(family, precision, workload, table="traffic.json"):
    """The committed counter summary of the `family` kernel running
    `precision` on `workload` (profiles/<table>, key family:precision:workload),
    or None when there is none or the kernel's sources changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", table)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        entry = json.load(fh).get("kernels", {}).get(f"{family}:{precision}:{workload}")
    if not entry or entry.get("sources_sha256") != sources_sha256(family):
        return None
    return entry


def counter_traffic(family, precision, workload):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter runs
    (scaled by the plain-copy calibration), or None."""
    e = counter_entry(family, precision, workload)
    return None if e is None else e["bytes_per_launch"]


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
        KS = 1 if N <= 64 else (2 if N <= 128 else (4 if N <= 192 else 8))
        NK = N // KS
        M1 = P * ((R + 3) // 4 * 4)
        per_c = KS * (-(-M1 // 16) * (2 * NK // 16) * KK + (N // 16) * (NK // 16) * P * 2 * KK)
        total += int(per_c.sum())
    return total


def grid_mfma_per_call(info, subs, T):
    """MFMA 16x16x32 instructions of the gridding product of a GEMM-gridding
    plan: per column part and channel, each block entry is multiplied once per
    step of grid_step spectra and per split term (FP16 2, FP8 3)."""
    total = 0
    for k, s in enumerate(subs):
        if info["grid_form"][k] == 1:
            continue
        terms = 3 if info["precision"] == 2 else 2
        steps = -(-T // info["grid_step"][k])
        total += info["col_split"][k] * info["grid_blocks"][k] * terms * steps
    return total


def mfma_fraction(info, kern_ms):
    """Executed MFMA rate of a matrix-core call against the dense peaks: the
    FP16 transform products, and the gridding product (FP16 or FP8)."""
    ops = info["mfma_ops_per_call"]
    gops = info.get("grid_mfma_per_call", 0)
    t_tf = ops * MFMA_FLOPS / (kern_ms * 1e-3) / 1e12
    t_g = gops * MFMA_FLOPS / (kern_ms * 1e-3) / 1e12
    gpeak = FP8_MFMA_PEAK_TFLOPS if info["precision"] == 2 else FP16_MFMA_PEAK_TFLOPS
    return {"executed_ops_per_call": ops, "executed_tflops": t_tf, "peak": FP16_MFMA_PEAK_TFLOPS,
            "frac": t_tf / FP16_MFMA_PEAK_TFLOPS, "grid_ops_per_call": gops, "grid_tflops": t_g,
            "grid_peak": gpeak, "frac_total": t_tf / FP16_MFMA_PEAK_TFLOPS + t_g / gpeak,
            "source": "tile counts of the plan's shapes (transforms: counter-checked)"}


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


def cpu_baseline(sub, samples, budget_s=30.0):
    """Time the FP64 oracle on the workload: all channels over the first T_s
    spectra, every spectrum when that fits ~budget_s of wall time (the station
    does, in ~15 s on 16 cores).  Returns the JSON record and the oracle's
    image of those spectra, the reference of the parity figures."""
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    probe_t = 4
    t0 = time.perf_counter()
    oracle.image(sub, samples[:probe_t], n_threads=cores)
    dt = time.perf_counter() - t0
    T_s = int(max(probe_t, min(samples.shape[0], budget_s / max(dt, 1e-6) * probe_t)))
    t0 = time.perf_counter()
    ref = oracle.image(sub, samples[:T_s], n_threads=cores)
    wall = time.perf_counter() - t0
    n = sub.n_ant * sub.n_pol * sub.n_chan * T_s
    rec = {"value": n / wall, "unit": "samples/s", "cores": cores, "kind": "oracle",
           "sample": f"all {sub.n_chan} channels x {'all' if T_s == samples.shape[0] else 'first'} {T_s} of "
                     f"{samples.shape[0]} spectra ({wall:.1f} s wall, FP64 C loops, OpenMP over channels)"}
    return rec, ref, T_s


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


def run_sweep(kind, steps, warmup):
    """The paper's measurement axes (Sec. 3.1 and 3.2, Figs. 3 and 4): time per
    accumulate call of the station shape against the channel count at 64 x 64
    (1000 spectra), and against the grid size at 4 channels, for the FP32 form
    and the FP16 matrix-core form.  The work does not depend on the sample
    values, so the inputs are uniform random bytes drawn on the device."""
    import dataclasses

    import torch
    from paper_2301_09662_amd import epic as E

    base = synth.workload(2).subs[0]
    T = 1000
    if kind == "channels":
        shapes = [(dataclasses.replace(base, n_chan=c), {"n_chan": c, "grid_n": base.grid_n})
                  for c in (1, 2, 4, 8, 16, 33, 66, 132)]
    else:
        shapes = [(dataclasses.replace(base, n_chan=4, grid_n=n), {"n_chan": 4, "grid_n": n})
                  for n in (32, 48, 64, 96, 128, 192, 256)]
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device=dev)
    gen.manual_seed(230109662)
    points = []
    for sub, key in shapes:
        x = torch.randint(0, 256, (T, sub.n_chan, sub.n_ant, sub.n_pol), dtype=torch.uint8, device=dev,
                          generator=gen)
        pt = dict(key)
        for prec in ("fp32", "fp16"):
            plan = E.epic_plan([sub], precision=prec, max_time=T, gridder="gather")
            try:
                info = E.epic_plan_query(plan)
                out = torch.empty((sub.n_chan, info["npp"][0], sub.grid_n, sub.grid_n), device=dev)
                ms = []
                for k in range(warmup + steps):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    E.epic_grid_fft_accumulate(plan, [x], T, stream)
                    b.record(stream)
                    E.epic_readout(plan, [out], 1, stream)
                    torch.cuda.synchronize()
                    if k >= warmup:
                        ms.append(a.elapsed_time(b))
            finally:
                E.epic_destroy(plan)
            med = float(np.median(ms))
            pt[f"{prec}_ms"] = med
            pt[f"{prec}_samples_per_s"] = sub.n_ant * sub.n_pol * sub.n_chan * T / (med * 1e-3)
            pt[f"{prec}_tflops"] = algorithmic_flops_per_ct(sub) * sub.n_chan * T / (med * 1e-3) / 1e12
        pt["fp16_speedup"] = pt["fp32_ms"] / pt["fp16_ms"]
        points.append(pt)
    print(json.dumps({"sweep": kind, "workload": "station layout (256 ant x 2 pol, dl = 1), 1000 spectra per "
                      "call, accumulate kernel time (HIP events, median)", "steps": steps, "warmup": warmup,
                      "points": points}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cfg", type=int, default=2, help="workload config (default: station FP32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reduced", action="store_true", help="skip the reduced-precision legs")
    ap.add_argument("--legs", default="fp16:gather,fp16:block,fp16:dense,fp8:block",
                    help="reduced-precision legs of an FP32 workload, precision:gridder, comma-separated")
    ap.add_argument("--gridder", choices=["auto", "gather", "dense", "block", "direct"], default="auto",
                    help="gridding form of the workload's own run")
    ap.add_argument("--precision", choices=["fp32", "fp16", "fp8"], default=None,
                    help="override the workload's own precision")
    ap.add_argument("--no-graph", action="store_true", help="batched workloads: eager launches instead of graph replay")
    ap.add_argument("--sweep", choices=["channels", "grid"], default=None,
                    help="only time the station shape against the channel count (64 x 64) or the grid size "
                         "(4 channels), FP32 and FP16, and print one JSON line of points")
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
    if args.sweep:
        run_sweep(args.sweep, args.steps, args.warmup)
        return

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

    def run(precision, steps, warmup, flags=0, gridder="auto"):
        plan = E.epic_plan(subs, precision=precision, max_time=T, flags=flags, gridder=gridder)
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
        if precision != "fp32":
            info = dict(info, mfma_ops_per_call=mfma_ops_per_spectrum(plan, subs) * T,
                        grid_mfma_per_call=grid_mfma_per_call(info, subs, T))
        img = [o.double().cpu().numpy() for o in outs]
        if T_par is not None and T_par != T:     # the images the oracle's spectra give
            E.epic_grid_fft_accumulate(plan, [x[:T_par] for x in d_samples], T_par, stream)
            E.epic_readout(plan, outs, 1, stream)
            torch.cuda.synchronize()
            img = [o.double().cpu().numpy() for o in outs]
        E.epic_destroy(plan)
        return wall / steps * 1e3, kern_ms, img, info

    # the FP64 oracle first (timed on the host's cores): its image of the
    # first T_par spectra is the reference of every form's parity figures
    cpu = ref = None
    T_par = None
    if not args.no_cpu_baseline:
        cpu, ref, T_par = cpu_baseline(subs[0], host[0])

    def parity(img, prec):
        """Per-channel relative image error of sub-array 0 against the oracle."""
        if ref is None:
            return None
        e = rel_image_errors(img[0], ref).max(axis=1)
        return {"max": float(e.max()), "median": float(np.median(e)), "bar": TOL[prec],
                "ok": bool(e.max() <= TOL[prec]),
                "per_channel": [float(f"{v:.3g}") for v in e]}

    # each workload's own precision; the uneven batch of sub-arrays runs as
    # one autotuned persistent launch replayed from a hipGraph
    precision = args.precision or wl.precision
    flags = 0
    if len(subs) > 1:
        flags = E.EPIC_F_AUTOTUNE | (0 if args.no_graph else E.EPIC_F_GRAPH)
    ms_per_step, kern_ms, img32, info32 = run(precision, args.steps, args.warmup, flags, args.gridder)
    achieved = flops_per_launch / (kern_ms * 1e-3) / 1e12
    family = kernel_family(precision, info32)
    dtype = {"fp32": "f32", "fp16": "f16 operands, f32 accumulate",
             "fp8": "e4m3 gridding operands, f16 transforms, f32 accumulate"}[precision]
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
        "dtype": dtype,
        "data": "synthetic (seeded 4+4-bit noise + point sources, LWA-station shapes)",
        "config": {"workload": f"{wl.name}: " + "; ".join(
            f"{s.n_ant} ant x {s.n_pol} pol, {s.n_chan} ch, N={s.grid_n}, dl={s.grid_dl}" for s in subs)
            + f", T={T} spectra per step", "n_time": T, "precision": precision,
            "plan": {k: info32[k] for k in ("batched", "can_batch", "form_ms", "autotuned", "graph", "weight",
                                            "slots", "lds_bytes", "grid_form", "grid_step")}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": counter_traffic(family, precision, wl.name),
                     "kernel_ms": kern_ms, "algorithmic_flops_per_launch": flops_per_launch},
    }
    if res["roofline"]["traffic"] is not None:
        res["roofline"]["hbm_frac"] = res["roofline"]["traffic"] / (kern_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
    res["roofline"]["kernel_family"] = family
    valu = counter_entry(family, precision, wl.name, "valu.json")
    if valu is not None:
        # floating-point work the kernel executes, from the VALU instruction
        # counters (lanes x flop per instruction), at the measured time
        ex = valu["fp_flops_per_launch"] / (kern_ms * 1e-3) / 1e12
        res["roofline"]["executed_fp32"] = {"tflops": ex, "frac_of_peak": ex / FP32_PEAK_TFLOPS,
                                            "flops_per_launch": valu["fp_flops_per_launch"],
                                            "profile": valu["profile"]}
    if precision != "fp32":
        res["roofline"]["mfma"] = mfma_fraction(info32, kern_ms)
    par = {"reference": None if ref is None else
           f"FP64 oracle, all {subs[0].n_chan} channels x {T_par} spectra of sub-array 0"}
    par[f"{precision}:{args.gridder}"] = parity(img32, precision)
    if not args.no_reduced and precision == "fp32":
        legs = []
        for leg in [x for x in args.legs.split(",") if x]:
            lp, lg = leg.split(":")
            try:
                ms_l, kern_l, img_l, info_l = run(lp, args.steps, args.warmup, 0, lg)
            except E.EpicError as err:   # no kernel for this shape / form
                legs.append({"form": leg, "unavailable": str(err)})
                continue
            p = parity(img_l, lp)
            par[leg] = p
            fam_l = kernel_family(lp, info_l)
            tr_l = counter_traffic(fam_l, lp, wl.name)
            legs.append({"form": leg, "precision": lp, "gridder": lg, "grid_step": info_l["grid_step"],
                         "kernel_family": fam_l, "traffic": tr_l,
                         "hbm_frac": None if tr_l is None else tr_l / (kern_l * 1e-3) / (HBM_PEAK_GBS * 1e9),
                         "value": samples_per_step / (ms_l * 1e-3), "ms_per_step": ms_l, "kernel_ms": kern_l,
                         "speedup_vs_fp32": ms_per_step / ms_l,
                         "max_rel_image_err_vs_oracle": None if p is None else p["max"],
                         "achieved_algorithmic_tflops": flops_per_launch / (kern_l * 1e-3) / 1e12,
                         "mfma": mfma_fraction(info_l, kern_l)})
        ok = [x for x in legs if "value" in x and (x["max_rel_image_err_vs_oracle"] or 0.0) <= 1e-3]
        best = max(ok, key=lambda x: x["value"]) if ok else None
        res["reduced_precision"] = {"legs": legs, "best": None if best is None else best["form"],
                                    "best_speedup_vs_fp32": None if best is None else best["speedup_vs_fp32"]}
    res["parity"] = par
    if cpu is not None:
        res["cpu_baseline"] = cpu
        res["cpu_numpy_fft"] = cpu_numpy_fft(subs[0], host[0])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
