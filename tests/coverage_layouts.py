"""Hand-built antenna layouts whose aperture windows have chosen sizes, so
that the parity tests reach every compiled variant of the hot kernels.

The FP32 kernel folds each row of the aperture window (length W, the window's
x extent) and each column (length R, its y extent) in blocks of 8 before a
register 8-point DFT.  Grids up to 64 fold a row of two or three blocks with a
fixed-length routine specialised on the number of non-zero inputs of its last
block rounded up to 1, 2, 4 or 8; every other row and every column takes the
generic fold, whose last block has the same four tail branches and whose
middle-block loop runs from three blocks on.  The matrix-core kernel is
compiled per (grid side N, 32-deep step count KK), KK = ceil(window / 16)
with the window side rounded up to 8.  These helpers place a few antennas so
that one channel's window is exactly W x R cells, and classify windows the
way the kernels dispatch on them.

Layouts only: no imaging arithmetic lives here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

C0 = 299792458.0


@dataclass
class Box:
    """One sub-array, one channel, whose aperture window is W x R cells."""
    ant_xy: np.ndarray
    n_pol: int
    grid_n: int
    kernel_k: int = 3
    n_chan: int = 1
    grid_dl: float = 1.0
    freq0_hz: float = 40e6
    dfreq_hz: float = 0.0
    W: int = 0
    R: int = 0
    sources: List = field(default_factory=list)

    @property
    def n_ant(self) -> int:
        return int(self.ant_xy.shape[0])


def box(N: int, W: int, R: int, P: int = 2, K: int = 3, n_extra: int = 4, seed: int = 0) -> Box:
    """Antennas whose K x K footprints span exactly W x R cells, centred in an
    N x N grid at one wavelength per cell: two corner antennas plus n_extra
    inside, each at a random sub-cell offset of at most 0.4 cell."""
    hk = K // 2
    if W < K or R < K or W > N or R > N:
        raise ValueError("window must hold one footprint and fit the grid")
    rng = np.random.default_rng(seed)
    lam = C0 / 40e6
    x0, y0 = (N - W) // 2 + hk, (N - R) // 2 + hk          # nearest cells of the corner antennas
    x1, y1 = x0 + W - K, y0 + R - K
    cells = [(x0, y0), (x1, y1)]
    for _ in range(n_extra):
        cells.append((int(rng.integers(x0, x1 + 1)), int(rng.integers(y0, y1 + 1))))
    cells = np.array(cells, dtype=np.float64)
    frac = rng.uniform(-0.4, 0.4, cells.shape)
    xy = (cells - N / 2 + frac) * lam                      # g = x / lam + N / 2 at dl = 1
    return Box(xy, P, N, K, W=W, R=R)


# Windows (W, R) whose rows reach every fixed-length row fold (two and three
# blocks, tails 1, 2, 4, 8), the generic row fold with one and four blocks
# (all tails), and the generic column fold with one, two and three-plus
# blocks (all tails).
FOLD_WINDOWS = [(9, 5), (10, 9), (12, 10), (16, 11), (17, 15), (18, 17), (20, 18), (24, 20), (6, 21),
                (25, 25), (26, 26), (28, 28), (30, 30)]


def fold_class(length: int, fixed: bool):
    """(kind, blocks, tail class) of the fold a row or column of `length`
    non-zero inputs takes: kind 'fixed' for the fixed-length routine, else
    'generic' with blocks capped at 3 (the middle-block loop runs from 3 on)
    and the last block's tail rounded up to 1, 2, 4 or 8 (0: one block, no
    tail branch)."""
    nb = (length + 7) // 8
    tail = length - 8 * (nb - 1)
    last = 1 if tail <= 1 else 2 if tail <= 2 else 4 if tail <= 4 else 8
    if fixed and nb in (2, 3):
        return ("fixed", nb, last)
    return ("generic", min(nb, 3), last if nb >= 2 else 0)


ALL_FIXED = {("fixed", nb, last) for nb in (2, 3) for last in (1, 2, 4, 8)}
ALL_GENERIC = {("generic", 1, 0)} | {("generic", nb, last) for nb in (2, 3) for last in (1, 2, 4, 8)}


def windows_of(cells: np.ndarray, K: int):
    """(W, R) per channel from the nearest cells [C][A][2] (x, y)."""
    w = cells[:, :, 0].max(axis=1) - cells[:, :, 0].min(axis=1) + K
    r = cells[:, :, 1].max(axis=1) - cells[:, :, 1].min(axis=1) + K
    return w, r


# (N, KK, W, R): one window per matrix-core kernel shape.
MFMA_SHAPES = [(32, 1, 13, 9), (32, 2, 20, 29),
               (48, 1, 16, 12), (48, 2, 25, 31), (48, 3, 45, 40),
               (64, 1, 11, 14), (64, 2, 30, 18), (64, 3, 35, 44), (64, 4, 61, 50),
               (96, 1, 15, 10), (96, 2, 24, 32), (96, 3, 47, 33), (96, 4, 52, 63),
               (128, 1, 9, 16), (128, 2, 32, 30), (128, 3, 41, 48), (128, 4, 64, 57),
               (192, 1, 12, 15), (192, 2, 30, 20), (192, 3, 40, 45), (192, 4, 60, 55),
               (256, 1, 16, 10), (256, 2, 25, 32), (256, 3, 44, 37), (256, 4, 58, 63)]

# the shapes of the GEMM-gridding kernel (grids up to 128)
BGEMM_SHAPES = [s for s in MFMA_SHAPES if s[0] <= 128]

# the shapes the single persistent launch of several sub-arrays can run
BATCH_SHAPES = [s for s in MFMA_SHAPES if s[0] <= 96]


def kk_of(window_max: int) -> int:
    """32-deep MFMA steps for a window side (already rounded up to 8)."""
    return (window_max + 15) // 16
