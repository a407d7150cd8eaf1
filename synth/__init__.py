"""Seeded synthetic F-engine streams for the EPIC/MOFF imaging workloads.

This module is shared by the tests, the benchmark and the oracle's tests, and
deliberately holds none of the imaging arithmetic (no gridding, no transform,
no polarisation products).  It only produces what an F-engine would emit:

* antenna layouts (east, north metres) shaped like the station in Sec. 2.1
  (pseudo-random dipoles in a 110 m x 100 m ellipse) and the other arrays the
  workloads name;
* channel centre frequencies (25 kHz channels, Sec. 2.1);
* point sources on image-pixel centres, each antenna's field being the source
  signal times the plane-wave phase ``exp(-2 pi i (u l0 + v m0))`` of Eq. 1;
* complex Gaussian receiver noise;
* 4+4-bit quantisation (round half to even, clip to [-8, 7]) and packing into
  one byte per complex sample, real part in the high nibble by default
  (Sec. 2.1 names the 4+4-bit format; the nibble order is our reading).

Every random draw comes from ``numpy.random.SeedSequence([230109662, cfg])``
spawned into independent layout / source / noise streams, so a workload is a
pure function of its config number.  Sample layout is ``uint8[T][C][A][P]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

C0 = 299792458.0          # speed of light, m/s
ROOT_SEED = 230109662     # arXiv id of the paper
CHAN_BW_HZ = 25_000.0     # F-engine channel width (Sec. 2.1)


@dataclass
class Source:
    """A point source on an image-pixel centre (pixel indices i, j)."""
    i: int
    j: int
    sigma: float                 # per-component std of the source signal
    rho: float = 0.0             # Y = rho e^{i psi} X + sqrt(1-rho^2) X'
    psi: float = 0.0


@dataclass
class SubArray:
    name: str
    ant_xy: np.ndarray           # float64 [A][2], metres (east, north)
    n_pol: int
    n_chan: int
    grid_n: int
    grid_dl: float               # grid spacing in wavelengths
    freq0_hz: float
    dfreq_hz: float = CHAN_BW_HZ
    kernel_k: int = 3
    sources: List[Source] = field(default_factory=list)
    noise_sigma: float = 2.0
    seed_key: tuple = ()

    @property
    def n_ant(self) -> int:
        return int(self.ant_xy.shape[0])

    def freqs(self) -> np.ndarray:
        return self.freq0_hz + np.arange(self.n_chan, dtype=np.float64) * self.dfreq_hz

    def pixel_lm(self, i: int, j: int):
        """Direction cosines of pixel (i, j) (pixel N/2 is the phase centre)."""
        n, dl = self.grid_n, self.grid_dl
        return (i - n // 2) / (n * dl), (j - n // 2) / (n * dl)


@dataclass
class Workload:
    cfg: int
    name: str
    subs: List[SubArray]
    n_time: int
    precision: str               # "fp32" | "fp16" | "fp8"


# --------------------------------------------------------------------------
# layouts
# --------------------------------------------------------------------------

def layout_disk(rng: np.random.Generator, n: int, diameter_m: float) -> np.ndarray:
    r = 0.5 * diameter_m * np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def layout_ellipse(rng: np.random.Generator, n: int, width_x_m: float, width_y_m: float) -> np.ndarray:
    xy = layout_disk(rng, n, 2.0)  # unit disk
    return xy * np.array([0.5 * width_x_m, 0.5 * width_y_m])


def layout_jittered_square(rng: np.random.Generator, n: int, side_m: float) -> np.ndarray:
    """Square lattice of ceil(sqrt(n))^2 sites over ``side_m``, uniform jitter of
    +-pitch/4 on each axis, surplus sites dropped by a seeded permutation."""
    m = int(np.ceil(np.sqrt(n)))
    pitch = side_m / m
    c = -0.5 * side_m + pitch * (np.arange(m) + 0.5)
    gx, gy = np.meshgrid(c, c, indexing="xy")
    xy = np.stack([gx.ravel(), gy.ravel()], axis=1)
    xy = xy + rng.uniform(-0.25 * pitch, 0.25 * pitch, size=xy.shape)
    keep = np.sort(rng.permutation(xy.shape[0])[:n])
    return xy[keep]


def _pick_pixels(rng, n_src, grid_n, grid_dl, lm_max=0.35):
    lim = int(np.floor(lm_max * grid_n * grid_dl))
    out = []
    while len(out) < n_src:
        i = grid_n // 2 + int(rng.integers(-lim, lim + 1))
        j = grid_n // 2 + int(rng.integers(-lim, lim + 1))
        if (i, j) not in out:
            out.append((i, j))
    return out


def _sources(rng, sigmas, grid_n, grid_dl, polarised_first):
    pix = _pick_pixels(rng, len(sigmas), grid_n, grid_dl)
    srcs = []
    for k, (s, (i, j)) in enumerate(zip(sigmas, pix)):
        if k == 0 and polarised_first:
            srcs.append(Source(i, j, s, rho=0.6, psi=float(rng.uniform(-np.pi, np.pi))))
        else:
            srcs.append(Source(i, j, s))
    return srcs


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def _streams(cfg: int, sub: int = 0):
    ss = np.random.SeedSequence([ROOT_SEED, cfg, sub])
    lay, src, noise = ss.spawn(3)
    return (np.random.default_rng(lay), np.random.default_rng(src), (ROOT_SEED, cfg, sub))


def workload(cfg: int) -> Workload:
    """Config 1..5 of the benchmark suite (shapes of the paper's station workload).

    1  tiny single-pol FP32: 16 ant in a 20 m disk, 4 ch, N=32 at 0.5 lambda, T=64
    2  station FP32: 256 dual-pol ant, 110 x 100 m ellipse, 132 ch, N=64 at 1 lambda, T=1000
    3  = 2 in reduced precision (FP16 MFMA form)
    4  three uneven sub-arrays in one batched launch, T=250
    5  2048 dual-pol ant on a jittered 300 m square, 256 ch, N=128, T=125
    6  the station of 2 on a 256 x 256 grid at 0.5 lambda, 132 ch, T=100 (wide grid)
    """
    if cfg == 1:
        lay, src, key = _streams(1)
        xy = layout_disk(lay, 16, 20.0)
        s = SubArray("tiny", xy, 1, 4, 32, 0.5, 40e6, seed_key=key)
        s.sources = _sources(src, [2.0], 32, 0.5, False)
        return Workload(1, "tiny-fp32", [s], 64, "fp32")
    if cfg in (2, 3):
        lay, src, key = _streams(2)
        xy = layout_ellipse(lay, 256, 100.0, 110.0)
        s = SubArray("station", xy, 2, 132, 64, 1.0, 40e6, seed_key=key)
        s.sources = _sources(src, [1.0, 0.7, 0.5], 64, 1.0, True)
        return Workload(cfg, "station-fp32" if cfg == 2 else "station-fp16", [s], 1000,
                        "fp32" if cfg == 2 else "fp16")
    if cfg == 4:
        subs = []
        spec = [("A-ellipse", 256, 132, 64, 40e6, ("ellipse", 100.0, 110.0)),
                ("B-disk70", 128, 64, 48, 50e6, ("disk", 70.0)),
                ("C-disk200", 512, 32, 96, 60e6, ("disk", 200.0))]
        for k, (name, na, nc, n, f0, shape) in enumerate(spec):
            lay, src, key = _streams(4, k)
            if shape[0] == "ellipse":
                xy = layout_ellipse(lay, na, shape[1], shape[2])
            else:
                xy = layout_disk(lay, na, shape[1])
            s = SubArray(name, xy, 2, nc, n, 1.0, f0, seed_key=key)
            s.sources = _sources(src, [1.0, 0.7, 0.5], n, 1.0, True)
            subs.append(s)
        return Workload(4, "batched-3sub-fp16", subs, 250, "fp16")
    if cfg == 5:
        lay, src, key = _streams(5)
        xy = layout_jittered_square(lay, 2048, 300.0)
        s = SubArray("large", xy, 2, 256, 128, 1.0, 40e6, seed_key=key)
        s.sources = _sources(src, [1.0, 0.7, 0.5], 128, 1.0, True)
        return Workload(5, "large-2048ant", [s], 125, "fp8")
    if cfg == 6:
        lay, src, key = _streams(2)
        xy = layout_ellipse(lay, 256, 100.0, 110.0)
        s = SubArray("station-wide", xy, 2, 132, 256, 0.5, 40e6, seed_key=key)
        s.sources = _sources(src, [1.0, 0.7, 0.5], 256, 0.5, True)
        return Workload(6, "station-256grid", [s], 100, "fp32")
    raise ValueError(f"unknown config {cfg}")


def shrink(sub: SubArray, n_chan: Optional[int] = None, n_ant: Optional[int] = None) -> SubArray:
    """A smaller copy of a sub-array (first channels / first antennas), for
    parity cases the oracle finishes in seconds."""
    import copy
    s = copy.copy(sub)
    if n_chan is not None:
        s.n_chan = int(n_chan)
    if n_ant is not None:
        s.ant_xy = sub.ant_xy[: int(n_ant)].copy()
    return s


# --------------------------------------------------------------------------
# samples
# --------------------------------------------------------------------------

def quantise44(z: np.ndarray, nibble_order: int = 0) -> np.ndarray:
    """Round half to even, clip to [-8, 7] per component, pack two 4-bit
    two's-complement nibbles into one byte (real high by default)."""
    re = np.clip(np.rint(z.real), -8, 7).astype(np.int16)
    im = np.clip(np.rint(z.imag), -8, 7).astype(np.int16)
    hi, lo = (re, im) if nibble_order == 0 else (im, re)
    return (((hi & 0xF) << 4) | (lo & 0xF)).astype(np.uint8)


def pack44(re: np.ndarray, im: np.ndarray, nibble_order: int = 0) -> np.ndarray:
    """Pack integer components already in [-8, 7] (no rounding)."""
    re = np.asarray(re, dtype=np.int16)
    im = np.asarray(im, dtype=np.int16)
    if re.min(initial=0) < -8 or re.max(initial=0) > 7 or im.min(initial=0) < -8 or im.max(initial=0) > 7:
        raise ValueError("4-bit components must lie in [-8, 7]")
    hi, lo = (re, im) if nibble_order == 0 else (im, re)
    return (((hi & 0xF) << 4) | (lo & 0xF)).astype(np.uint8)


def samples(sub: SubArray, n_time: int, t0: int = 0, chan_chunk: int = 16) -> np.ndarray:
    """uint8[T][C][A][P] 4+4-bit stream for ``n_time`` spectra starting at ``t0``.

    Field of antenna a, pol p, channel c, time t:
        sum_k  s_k,p(t, c) exp(-2 pi i (u_a l_k + v_a m_k)) + noise,
    u_a = x_a f_c / c0, v_a = y_a f_c / c0.  Signals and noise are drawn per
    (t0 + t), so a window of a longer stream is reproducible on its own.
    """
    A, P, C = sub.n_ant, sub.n_pol, sub.n_chan
    out = np.empty((n_time, C, A, P), dtype=np.uint8)
    f = sub.freqs()
    ss = np.random.SeedSequence(list(sub.seed_key) + [7, t0, n_time])
    src_rng, noise_rng = [np.random.default_rng(s) for s in ss.spawn(2)]
    # per-source signals [T][C][P]
    sig = []
    for src in sub.sources:
        sx = src.sigma * (src_rng.standard_normal((n_time, C)) + 1j * src_rng.standard_normal((n_time, C)))
        if P == 2:
            sy_ind = src.sigma * (src_rng.standard_normal((n_time, C)) + 1j * src_rng.standard_normal((n_time, C)))
            sy = src.rho * np.exp(1j * src.psi) * sx + np.sqrt(1.0 - src.rho ** 2) * sy_ind
            sig.append(np.stack([sx, sy], axis=-1))
        else:
            sig.append(sx[..., None])
    for c0 in range(0, C, chan_chunk):
        c1 = min(C, c0 + chan_chunk)
        fc = f[c0:c1]
        z = sub.noise_sigma * (noise_rng.standard_normal((n_time, c1 - c0, A, P))
                               + 1j * noise_rng.standard_normal((n_time, c1 - c0, A, P)))
        for src, s in zip(sub.sources, sig):
            l0, m0 = sub.pixel_lm(src.i, src.j)
            u = sub.ant_xy[None, :, 0] * fc[:, None] / C0       # [c][a]
            v = sub.ant_xy[None, :, 1] * fc[:, None] / C0
            ph = np.exp(-2j * np.pi * (u * l0 + v * m0))          # [c][a]
            z += s[:, c0:c1, None, :] * ph[None, :, :, None]
        out[:, c0:c1] = quantise44(z)
    return out
