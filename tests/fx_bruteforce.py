"""FX-correlate-then-image brute force (paper Eq. 1-3), used only to pin the
oracle.

An FX correlator first forms visibilities V^{pq}_ab = sum_t E^p_a(t) E^q_b(t)*
(Eq. 1, here exact Gaussian integers), then images each baseline through the
product of the two antennas' kernel transforms.  By the MOFF identity (Eq. 3)
that image equals the EPIC image of Eq. 4 pixel by pixel, so this O(A^2 N^2)
route is an independent check of the oracle's O(N^3) gridding + DFT route.

The per-antenna kernel transform is evaluated directly at each pixel,
K^p_a(i, j) = sum over the antenna's taps of w (-1)^(x+y) exp(+2 pi i (x i + y j)/N),
from the geometry and taps the oracle exposes (its inputs, pinned separately).
"""
from __future__ import annotations

import numpy as np


def unpack_int(samples: np.ndarray, nibble_order: int = 0):
    """Integer (re, im) of packed 4+4-bit bytes via int8 shifts."""
    b = samples.astype(np.uint8)
    hi = (b.astype(np.int8) >> 4).astype(np.int64)
    lo = ((b << 4).astype(np.uint8).astype(np.int8) >> 4).astype(np.int64)
    return (hi, lo) if nibble_order == 0 else (lo, hi)


def kernel_images(cell_c: np.ndarray, taps_c: np.ndarray, N: int) -> np.ndarray:
    """complex128 [A][P][N][N] (indexed [j][i]) kernel transforms of one channel."""
    A, P, K, _ = taps_c.shape
    h = K // 2
    idx = np.arange(N)
    out = np.zeros((A, P, N, N), dtype=np.complex128)
    for dy in range(-h, h + 1):
        for dx in range(-h, h + 1):
            x = cell_c[:, 0] + dx
            y = cell_c[:, 1] + dy
            sgn = np.where((x + y) % 2 == 0, 1.0, -1.0)
            ph_x = np.exp(2j * np.pi * np.outer(x, idx) / N)   # [A][i]
            ph_y = np.exp(2j * np.pi * np.outer(y, idx) / N)   # [A][j]
            w = taps_c[:, :, dy + h, dx + h] * sgn[:, None]      # [A][P]
            out += w[:, :, None, None] * ph_y[:, None, :, None] * ph_x[:, None, None, :]
    return out


def fx_image(samples: np.ndarray, cell: np.ndarray, taps: np.ndarray, N: int,
             chans=None, nibble_order: int = 0, drop_auto: bool = False) -> np.ndarray:
    """FP64 [C][NPP][N][N] image via visibilities and direct per-pixel imaging.
    ``drop_auto`` leaves out the a = b baselines (each antenna with itself)."""
    T, C, A, P = samples.shape
    npp = 4 if P == 2 else 1
    chans = range(C) if chans is None else chans
    out = np.zeros((C, npp, N, N))
    re, im = unpack_int(samples, nibble_order)
    E = re + 1j * im                                           # exact small ints
    for c in chans:
        e = E[:, c]                                            # [T][A][P]
        Kc = kernel_images(cell[c], taps[c], N).reshape(A, P, N * N)
        def img(p, q):
            V = np.einsum("ta,tb->ab", e[:, :, p], np.conj(e[:, :, q]))   # Eq. 1
            if drop_auto:
                np.fill_diagonal(V, 0)
            M = V @ np.conj(Kc[:, q])                                      # [a][pix]
            return np.einsum("ap,ap->p", Kc[:, p], M).reshape(N, N)
        xx = img(0, 0)
        out[c, 0] = xx.real
        if P == 2:
            out[c, 1] = img(1, 1).real
            xy = img(0, 1)
            out[c, 2] = xy.real
            out[c, 3] = xy.imag
    return out
