"""FP64 CPU oracle of the EPIC/MOFF image -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it, and
it shares no code with the GPU path.  The arithmetic lives in
``epic_oracle.c`` (plain loops, FP64, no fused multiply-add); this module only
builds that file with gcc and marshals arguments through ctypes.

Functions follow paper Sec. 2 (Eq. 4) and Sec. 3.2 (Eq. 5); see the C file's
header for the readings it fixes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "epic_oracle.c")
_LIB = os.path.join(_HERE, "libepic_oracle.so")

ORA_OK, ORA_E_ARG, ORA_E_GEOMETRY, ORA_E_NOMEM = 0, 1, 2, 3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _OraArray(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("n_pol", ctypes.c_int32), ("n_chan", ctypes.c_int32),
                ("grid_n", ctypes.c_int32), ("kernel_k", ctypes.c_int32), ("nibble_order", ctypes.c_int32),
                ("grid_dl", ctypes.c_double), ("freq0_hz", ctypes.c_double), ("dfreq_hz", ctypes.c_double),
                ("kernel_sigma_cells", ctypes.c_double),
                ("ant_xy", ctypes.POINTER(ctypes.c_double)), ("taps", ctypes.POINTER(ctypes.c_float))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.ora_unpack_table.argtypes = [ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double)]
        lib.ora_geometry.argtypes = [P(_OraArray), P(ctypes.c_int32), P(ctypes.c_double)]
        lib.ora_taps.argtypes = [P(_OraArray), P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double)]
        lib.ora_grid.argtypes = [P(_OraArray), P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_uint8),
                                 ctypes.c_int, P(ctypes.c_double)]
        lib.ora_dft2.argtypes = [ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double)]
        lib.ora_image_range.argtypes = [P(_OraArray), P(ctypes.c_uint8), ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_int, P(ctypes.c_double), ctypes.c_int]
        lib.ora_autocorr_range.argtypes = lib.ora_image_range.argtypes
        lib.ora_efield_range.argtypes = lib.ora_image_range.argtypes
        lib.ora_max_threads.argtypes = []
        for f in ("ora_unpack_table", "ora_geometry", "ora_taps", "ora_grid", "ora_dft2",
                  "ora_image_range", "ora_autocorr_range", "ora_efield_range", "ora_max_threads"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class ArraySpec:
    """Plain description of one sub-array (duck-types any object with the same
    attribute names, e.g. the synthetic generator's ``SubArray``)."""

    def __init__(self, sub, taps: Optional[np.ndarray] = None, nibble_order: int = 0,
                 kernel_sigma_cells: float = 0.5):
        self.ant_xy = np.ascontiguousarray(np.asarray(sub.ant_xy, dtype=np.float64))
        self.n_ant = int(self.ant_xy.shape[0])
        self.n_pol = int(sub.n_pol)
        self.n_chan = int(sub.n_chan)
        self.grid_n = int(sub.grid_n)
        self.kernel_k = int(getattr(sub, "kernel_k", 3))
        self.grid_dl = float(sub.grid_dl)
        self.freq0_hz = float(sub.freq0_hz)
        self.dfreq_hz = float(sub.dfreq_hz)
        self.nibble_order = int(nibble_order)
        self.kernel_sigma_cells = float(kernel_sigma_cells)
        self.taps = None if taps is None else np.ascontiguousarray(np.asarray(taps, dtype=np.float32))

    def c_struct(self) -> _OraArray:
        s = _OraArray()
        s.n_ant, s.n_pol, s.n_chan = self.n_ant, self.n_pol, self.n_chan
        s.grid_n, s.kernel_k, s.nibble_order = self.grid_n, self.kernel_k, self.nibble_order
        s.grid_dl, s.freq0_hz, s.dfreq_hz = self.grid_dl, self.freq0_hz, self.dfreq_hz
        s.kernel_sigma_cells = self.kernel_sigma_cells
        s.ant_xy = _ptr(self.ant_xy, ctypes.c_double)
        s.taps = _ptr(self.taps, ctypes.c_float) if self.taps is not None else ctypes.POINTER(ctypes.c_float)()
        return s

    @property
    def npp(self) -> int:
        return 4 if self.n_pol == 2 else 1


def _spec(sub, **kw) -> ArraySpec:
    return sub if isinstance(sub, ArraySpec) else ArraySpec(sub, **kw)


def unpack_table(nibble_order: int = 0):
    """(re[256], im[256]) of every byte code."""
    lib = _load()
    re = np.zeros(256); im = np.zeros(256)
    lib.ora_unpack_table(int(nibble_order), _ptr(re, ctypes.c_double), _ptr(im, ctypes.c_double))
    return re, im


def geometry(sub, **kw):
    """(cell int32[C][A][2], g float64[C][A][2]) nearest cell and fractional cell
    coordinate (x then y); raises OracleError(2) if a footprint leaves the grid."""
    s = _spec(sub, **kw)
    lib = _load()
    cell = np.zeros((s.n_chan, s.n_ant, 2), dtype=np.int32)
    g = np.zeros((s.n_chan, s.n_ant, 2), dtype=np.float64)
    st = s.c_struct()
    rc = lib.ora_geometry(ctypes.byref(st), _ptr(cell, ctypes.c_int32), _ptr(g, ctypes.c_double))
    if rc:
        raise OracleError(rc, "geometry")
    return cell, g


def taps(sub, **kw) -> np.ndarray:
    """complex128 [C][A][P][K][K] gridding-kernel taps."""
    s = _spec(sub, **kw)
    lib = _load()
    cell, g = geometry(s)
    K = s.kernel_k
    out = np.zeros((s.n_chan, s.n_ant, s.n_pol, K, K, 2), dtype=np.float64)
    st = s.c_struct()
    rc = lib.ora_taps(ctypes.byref(st), _ptr(cell, ctypes.c_int32), _ptr(g, ctypes.c_double),
                      _ptr(out, ctypes.c_double))
    if rc:
        raise OracleError(rc, "taps")
    return out[..., 0] + 1j * out[..., 1]


def grid(sub, samples: np.ndarray, t: int, c: int, p: int, **kw) -> np.ndarray:
    """complex128 [N][N] gridded aperture (with the (-1)^(x+y) factor) of one
    (t, c, p), indexed [y][x]."""
    s = _spec(sub, **kw)
    lib = _load()
    cell, g = geometry(s)
    tp = taps(s)
    tp_c = np.ascontiguousarray(np.stack([tp[c].real, tp[c].imag], axis=-1))
    cell_c = np.ascontiguousarray(cell[c])
    row = np.ascontiguousarray(samples[t, c])
    out = np.zeros((s.grid_n, s.grid_n, 2))
    st = s.c_struct()
    lib.ora_grid(ctypes.byref(st), _ptr(tp_c, ctypes.c_double), _ptr(cell_c, ctypes.c_int32),
                 _ptr(row, ctypes.c_uint8), int(p), _ptr(out, ctypes.c_double))
    return out[..., 0] + 1j * out[..., 1]


def dft2(x: np.ndarray) -> np.ndarray:
    """Unnormalised 2D DFT with exp(+2 pi i (x i + y j)/N) of a square complex
    array indexed [y][x]; result indexed [j][i]."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    lib = _load()
    a = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1))
    out = np.zeros_like(a)
    rc = lib.ora_dft2(int(n), _ptr(a, ctypes.c_double), _ptr(out, ctypes.c_double))
    if rc:
        raise OracleError(rc, "dft2")
    return out[..., 0] + 1j * out[..., 1]


def image(sub, samples: np.ndarray, chans: Optional[range] = None, n_threads: int = 0,
          remove_autocorr: bool = False, **kw) -> np.ndarray:
    """FP64 image cube [C][NPP][N][N] (products XX*, YY*, Re XY*, Im XY*; single
    pol: XX*), summed over all T spectra of ``samples`` (uint8 [T][C][A][P]).
    ``chans`` restricts the channels computed (others are returned as zero).
    ``remove_autocorr`` subtracts every antenna's own (a = b) contribution,
    which autocorr() returns."""
    out = _run("ora_image_range", sub, samples, chans, n_threads, **kw)
    if remove_autocorr:
        out -= _run("ora_autocorr_range", sub, samples, chans, n_threads, **kw)
    return out


def autocorr(sub, samples: np.ndarray, chans: Optional[range] = None, n_threads: int = 0, **kw) -> np.ndarray:
    """FP64 [C][NPP][N][N]: the a = b terms of the image, sum over antennas of
    K^p_a K^q_a^* sum_t E^p_a E^q_a^* (K^p_a: antenna a's kernel transformed alone)."""
    return _run("ora_autocorr_range", sub, samples, chans, n_threads, **kw)


def efield(sub, samples: np.ndarray, chans: Optional[range] = None, n_threads: int = 0, **kw) -> np.ndarray:
    """complex128 [T][C][P][N][N]: each spectrum's transformed field per
    polarisation (steps 1-3, before the products); channels outside ``chans``
    are zero."""
    s = _spec(sub, **kw)
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.uint8)
    T = samples.shape[0]
    if samples.shape[1:] != (s.n_chan, s.n_ant, s.n_pol):
        raise ValueError(f"samples shape {samples.shape} does not match the array")
    N = s.grid_n
    out = np.zeros((T, s.n_chan, s.n_pol, N, N, 2), dtype=np.float64)
    c0, c1 = (0, s.n_chan) if chans is None else (chans.start, chans.stop)
    st = s.c_struct()
    rc = lib.ora_efield_range(ctypes.byref(st), _ptr(samples, ctypes.c_uint8), int(T), int(c0), int(c1),
                              _ptr(out, ctypes.c_double), int(n_threads))
    if rc:
        raise OracleError(rc, "ora_efield_range")
    return out[..., 0] + 1j * out[..., 1]


def _run(fn, sub, samples, chans, n_threads, **kw):
    s = _spec(sub, **kw)
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.uint8)
    T = samples.shape[0]
    if samples.shape[1:] != (s.n_chan, s.n_ant, s.n_pol):
        raise ValueError(f"samples shape {samples.shape} does not match the array")
    N = s.grid_n
    out = np.zeros((s.n_chan, s.npp, N, N), dtype=np.float64)
    c0, c1 = (0, s.n_chan) if chans is None else (chans.start, chans.stop)
    st = s.c_struct()
    rc = getattr(lib, fn)(ctypes.byref(st), _ptr(samples, ctypes.c_uint8), int(T), int(c0), int(c1),
                          _ptr(out, ctypes.c_double), int(n_threads))
    if rc:
        raise OracleError(rc, fn)
    return out


def max_threads() -> int:
    return int(_load().ora_max_threads())


class using_library:
    """Context manager that points this wrapper at another build of the oracle
    source (the tests use it to check that a planted mistake fails a pin)."""

    def __init__(self, path: str):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = None
        keep = globals()["_LIB"]
        globals()["_LIB"] = self.path
        try:
            _load()
        finally:
            globals()["_LIB"] = keep
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def source_path() -> str:
    return _SRC
