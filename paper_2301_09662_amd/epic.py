"""Thin Python binding of the C ABI in ``include/epic.h`` (ctypes).

The functions keep the C names and only marshal arguments: every step of the
imaging path runs in ``libepic.so``'s HIP kernels.  Device buffers are torch
tensors (``data_ptr()``), streams are torch streams or raw ``hipStream_t``
integers.  If the library has not been built this module raises on import --
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

# torch ships its own HIP runtime under the same soname; loading it first makes
# this library bind to that one runtime, so torch's streams and allocations are
# valid handles here (two runtimes in one process do not share streams).
import torch  # noqa: F401  (imported for its HIP runtime)

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libepic.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "or `python -m paper_2301_09662_amd._build` (no CPU fallback exists)")
_lib = ctypes.CDLL(_LIB_PATH)

# ---- enums (include/epic.h) ------------------------------------------------
EPIC_OK, EPIC_E_ARG, EPIC_E_GEOMETRY, EPIC_E_NOMEM, EPIC_E_DEVICE, EPIC_E_UNSUPPORTED, EPIC_E_STATE = range(7)
EPIC_FP32, EPIC_FP16, EPIC_FP8 = 0, 1, 2
EPIC_GRID_AUTO, EPIC_GRID_GATHER, EPIC_GRID_DENSE_GEMM, EPIC_GRID_BLOCK_GEMM, EPIC_GRID_DIRECT_GEMM = 0, 1, 2, 3, 4
EPIC_OUT_POL, EPIC_OUT_STOKES = 0, 1
EPIC_F_GRAPH, EPIC_F_AUTOTUNE, EPIC_F_DRY_RUN, EPIC_F_REMOVE_AUTOCORR, EPIC_F_COMPLEX_WEIGHTS = 1, 2, 4, 8, 16
EPIC_F_ONE_LAUNCH = 32
PRECISIONS = {"fp32": EPIC_FP32, "fp16": EPIC_FP16, "fp8": EPIC_FP8}
GRIDDERS = {"auto": EPIC_GRID_AUTO, "gather": EPIC_GRID_GATHER, "dense": EPIC_GRID_DENSE_GEMM,
            "block": EPIC_GRID_BLOCK_GEMM, "direct": EPIC_GRID_DIRECT_GEMM}


class EpicError(RuntimeError):
    def __init__(self, status: int, call: str):
        super().__init__(f"{call}: {epic_status_str(status)}")
        self.status = status


class epic_array_desc(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("n_pol", ctypes.c_int32), ("n_chan", ctypes.c_int32),
                ("grid_n", ctypes.c_int32), ("kernel_k", ctypes.c_int32), ("nibble_order", ctypes.c_int32),
                ("grid_dl", ctypes.c_double), ("freq0_hz", ctypes.c_double), ("dfreq_hz", ctypes.c_double),
                ("ant_xy_m", ctypes.POINTER(ctypes.c_double)), ("taps", ctypes.POINTER(ctypes.c_float)),
                ("kernel_sigma_cells", ctypes.c_double)]


class epic_plan_desc(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("sub", ctypes.POINTER(epic_array_desc)),
                ("precision", ctypes.c_int32), ("gridder", ctypes.c_int32), ("output", ctypes.c_int32),
                ("device", ctypes.c_int32), ("max_time", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32 * 4)]


class epic_plan_info(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("precision", ctypes.c_int32), ("gridder", ctypes.c_int32),
                ("output", ctypes.c_int32), ("npp", ctypes.c_int32 * 16), ("slots", ctypes.c_int32 * 16),
                ("window_max", ctypes.c_int32 * 16), ("threads", ctypes.c_int32 * 16),
                ("device_bytes", ctypes.c_int64), ("lds_bytes", ctypes.c_int64 * 16),
                ("graph", ctypes.c_int32), ("autotuned", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("weight", ctypes.c_int32 * 16), ("col_split", ctypes.c_int32 * 16),
                ("workgroups", ctypes.c_int32 * 16), ("can_batch", ctypes.c_int32),
                ("form_ms", ctypes.c_double * 2), ("grid_form", ctypes.c_int32 * 16),
                ("grid_step", ctypes.c_int32 * 16), ("graph_builds", ctypes.c_int32),
                ("autocorr_pending", ctypes.c_int32 * 16), ("autocorr_fold_limit", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int64 * 16)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_lib.epic_plan.argtypes = [_P(epic_plan_desc), _vp, _P(_vp)]
_lib.epic_grid_fft_accumulate.argtypes = [_vp, _P(_vp), ctypes.c_int64, _vp]
_lib.epic_readout.argtypes = [_vp, _P(_vp), ctypes.c_int32, _vp]
_lib.epic_image_noalloc.argtypes = [_vp, _P(_vp), ctypes.c_int64, _P(_vp), _vp]
_lib.epic_set_gains.argtypes = [_vp, ctypes.c_int32, _P(ctypes.c_float), _vp]
_lib.epic_efield.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp]
_lib.epic_plan_query.argtypes = [_vp, _P(epic_plan_info)]
_lib.epic_debug_geometry.argtypes = [_vp, ctypes.c_int32, _P(ctypes.c_int32)]
_lib.epic_debug_schedule.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, _P(ctypes.c_int32), _P(ctypes.c_int32)]
_lib.epic_debug_unpack.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp]
_lib.epic_destroy.argtypes = [_vp]
_lib.epic_status_str.argtypes = [ctypes.c_int]
_lib.epic_status_str.restype = ctypes.c_char_p
_lib.epic_abi_version.argtypes = []
for _f in ("epic_plan", "epic_grid_fft_accumulate", "epic_readout", "epic_image_noalloc", "epic_set_gains", "epic_efield", "epic_plan_query",
           "epic_debug_geometry", "epic_debug_schedule", "epic_debug_unpack", "epic_destroy", "epic_abi_version"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("epic_plan", "epic_grid_fft_accumulate", "epic_readout", "epic_image_noalloc", "epic_set_gains", "epic_efield", "epic_plan_query",
            "epic_debug_geometry", "epic_debug_schedule", "epic_debug_unpack", "epic_destroy", "epic_status_str",
            "epic_abi_version")


def library_path() -> str:
    return _LIB_PATH


def epic_status_str(status: int) -> str:
    return _lib.epic_status_str(int(status)).decode()


def epic_abi_version() -> int:
    return int(_lib.epic_abi_version())


def _check(status: int, call: str):
    if status != EPIC_OK:
        raise EpicError(status, call)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t) -> int:
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("device buffer expected (a CUDA/HIP torch tensor)")
    if not t.is_contiguous():
        raise ValueError("device buffer must be contiguous")
    return t.data_ptr()


def _check_buffer(t, dtype: str, count: int, what: str):
    """A tensor argument must hold at least ``count`` elements of ``dtype``
    (raw device addresses are taken as they are: their size is the caller's
    responsibility, as in the C ABI)."""
    if isinstance(t, int):
        return
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{what}: {dtype} tensor expected, got {t.dtype}")
    if t.numel() < count:
        raise ValueError(f"{what}: {count} elements needed, tensor has {t.numel()}")


def _npp(plan, s) -> int:
    return 4 if int(s.n_pol) == 2 else 1


class Plan:
    """Owns an ``epic_plan_t`` handle and the host copies kept alive for it."""

    def __init__(self, handle: int, subs, keep):
        self.handle = handle
        self.subs = subs
        self._keep = keep

    def __int__(self):
        return self.handle

    @property
    def _as_parameter_(self):
        return ctypes.c_void_p(self.handle)


def _make_desc(sub, taps=None, nibble_order=0, kernel_sigma_cells=0.0):
    xy = np.ascontiguousarray(np.asarray(sub.ant_xy, dtype=np.float64))
    d = epic_array_desc()
    d.n_ant = int(xy.shape[0])
    d.n_pol = int(sub.n_pol)
    d.n_chan = int(sub.n_chan)
    d.grid_n = int(sub.grid_n)
    d.kernel_k = int(getattr(sub, "kernel_k", 3))
    d.nibble_order = int(nibble_order)
    d.grid_dl = float(sub.grid_dl)
    d.freq0_hz = float(sub.freq0_hz)
    d.dfreq_hz = float(sub.dfreq_hz)
    d.ant_xy_m = xy.ctypes.data_as(_P(ctypes.c_double))
    keep = [xy]
    if taps is not None:
        tp = np.ascontiguousarray(np.asarray(taps, dtype=np.float32))
        d.taps = tp.ctypes.data_as(_P(ctypes.c_float))
        keep.append(tp)
    else:
        d.taps = _P(ctypes.c_float)()
    d.kernel_sigma_cells = float(kernel_sigma_cells)
    return d, keep


def epic_plan(subs: Sequence, precision=EPIC_FP32, gridder=EPIC_GRID_AUTO, output=EPIC_OUT_POL, device: int = 0,
              max_time: int = 1, flags: int = 0, stream=None, taps: Optional[Sequence] = None,
              nibble_order: int = 0, kernel_sigma_cells: float = 0.0, reserved=(0, 0, 0, 0)) -> Plan:
    """Create a plan for ``subs`` (objects with ant_xy, n_pol, n_chan, grid_n,
    grid_dl, freq0_hz, dfreq_hz, kernel_k)."""
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    if isinstance(gridder, str):
        gridder = GRIDDERS[gridder]
    n = len(subs)
    arr = (epic_array_desc * max(n, 1))()
    keep = []
    for k, s in enumerate(subs):
        d, kp = _make_desc(s, None if taps is None else taps[k], nibble_order, kernel_sigma_cells)
        arr[k] = d
        keep += kp
    pd = epic_plan_desc()
    pd.n_sub, pd.sub = n, ctypes.cast(arr, _P(epic_array_desc))
    pd.precision, pd.gridder, pd.output = int(precision), int(gridder), int(output)
    pd.device, pd.max_time, pd.flags = int(device), int(max_time), int(flags)
    for k in range(4):
        pd.reserved[k] = int(reserved[k])
    h = _vp()
    dry = bool(flags & EPIC_F_DRY_RUN)
    st = None if dry else _stream_handle(stream)
    _check(_lib.epic_plan(ctypes.byref(pd), st, ctypes.byref(h)), "epic_plan")
    return Plan(h.value, list(subs), keep)


def epic_grid_fft_accumulate(plan: Plan, samples: Sequence, n_time: int, stream=None):
    """Enqueue the hot path on ``stream``; ``samples[s]`` is a uint8 device
    tensor [n_time][C][A][P] (or a raw device address)."""
    if len(samples) != len(plan.subs):
        raise ValueError(f"one sample buffer per sub-array expected ({len(plan.subs)}), got {len(samples)}")
    for k, (t, s) in enumerate(zip(samples, plan.subs)):
        _check_buffer(t, "uint8", int(n_time) * int(s.n_chan) * int(np.asarray(s.ant_xy).shape[0]) * int(s.n_pol),
                      f"samples[{k}]")
    ptrs = (_vp * max(len(samples), 1))(*[_dev_ptr(t) for t in samples])
    _check(_lib.epic_grid_fft_accumulate(plan, ptrs, int(n_time), _stream_handle(stream)),
           "epic_grid_fft_accumulate")


def epic_readout(plan: Plan, images: Sequence, reset: int = 0, stream=None):
    """Reduce the accumulators into ``images[s]`` (float32 device tensors
    [C][NPP][N][N]); zero them afterwards if ``reset``."""
    if len(images) != len(plan.subs):
        raise ValueError(f"one image cube per sub-array expected ({len(plan.subs)}), got {len(images)}")
    for k, (t, s) in enumerate(zip(images, plan.subs)):
        _check_buffer(t, "float32", int(s.n_chan) * _npp(plan, s) * int(s.grid_n) ** 2, f"images[{k}]")
    ptrs = (_vp * max(len(images), 1))(*[_dev_ptr(t) for t in images])
    _check(_lib.epic_readout(plan, ptrs, int(reset), _stream_handle(stream)), "epic_readout")


NOALLOC_MAX_BYTES = 64 << 20   # EPIC_NOALLOC_MAX_BYTES


def epic_image_noalloc(plan: Plan, samples: Sequence, n_time: int, images: Sequence, stream=None):
    """One integration of ``n_time`` spectra straight into ``images[s]``
    (float32 device tensors [C][NPP][N][N]) with the library's static scratch
    instead of the plan's accumulators; allocates no device memory."""
    if len(samples) != len(plan.subs) or len(images) != len(plan.subs):
        raise ValueError(f"one sample buffer and one image cube per sub-array expected ({len(plan.subs)})")
    for k, (x, y, s) in enumerate(zip(samples, images, plan.subs)):
        _check_buffer(x, "uint8", int(n_time) * int(s.n_chan) * int(np.asarray(s.ant_xy).shape[0]) * int(s.n_pol),
                      f"samples[{k}]")
        _check_buffer(y, "float32", int(s.n_chan) * _npp(plan, s) * int(s.grid_n) ** 2, f"images[{k}]")
    xp = (_vp * max(len(samples), 1))(*[_dev_ptr(t) for t in samples])
    yp = (_vp * max(len(images), 1))(*[_dev_ptr(t) for t in images])
    _check(_lib.epic_image_noalloc(plan, xp, int(n_time), yp, _stream_handle(stream)), "epic_image_noalloc")


def epic_set_gains(plan: Plan, sub: int, gains: Optional[np.ndarray], stream=None):
    """Per-antenna complex gains of sub-array ``sub``: host float32
    [C][A][P][2] (re, im), or None for unit gains."""
    g = None if gains is None else np.ascontiguousarray(np.asarray(gains, dtype=np.float32))
    if g is not None and 0 <= int(sub) < len(plan.subs):
        s = plan.subs[int(sub)]
        n = int(s.n_chan) * int(np.asarray(s.ant_xy).shape[0]) * int(s.n_pol) * 2
        if g.size != n:
            raise ValueError(f"gains: {n} floats ([C][A][P][2]) expected, got {g.size}")
    ptr = _P(ctypes.c_float)() if g is None else g.ctypes.data_as(_P(ctypes.c_float))
    _check(_lib.epic_set_gains(plan, int(sub), ptr, _stream_handle(stream)), "epic_set_gains")


def epic_efield(plan: Plan, sub: int, samples, n_time: int, out, stream=None):
    """E-field images of sub-array ``sub``: ``out`` is a float32 device tensor
    [n_time][C][P][N][N][2] (or a raw device address)."""
    if 0 <= int(sub) < len(plan.subs):
        s = plan.subs[int(sub)]
        A = int(np.asarray(s.ant_xy).shape[0])
        _check_buffer(samples, "uint8", int(n_time) * int(s.n_chan) * A * int(s.n_pol), "samples")
        _check_buffer(out, "float32", int(n_time) * int(s.n_chan) * int(s.n_pol) * int(s.grid_n) ** 2 * 2, "out")
    _check(_lib.epic_efield(plan, int(sub), _dev_ptr(samples), int(n_time), _dev_ptr(out), _stream_handle(stream)),
           "epic_efield")


def epic_plan_query(plan: Plan) -> dict:
    info = epic_plan_info()
    _check(_lib.epic_plan_query(plan, ctypes.byref(info)), "epic_plan_query")
    n = info.n_sub
    return {"n_sub": n, "precision": info.precision, "gridder": info.gridder, "output": info.output,
            "npp": list(info.npp[:n]), "slots": list(info.slots[:n]), "window_max": list(info.window_max[:n]),
            "threads": list(info.threads[:n]), "device_bytes": int(info.device_bytes),
            "lds_bytes": list(info.lds_bytes[:n]), "graph": info.graph, "autotuned": info.autotuned,
            "batched": info.batched, "weight": list(info.weight[:n]), "col_split": list(info.col_split[:n]),
            "workgroups": list(info.workgroups[:n]), "can_batch": info.can_batch,
            "form_ms": list(info.form_ms), "grid_form": list(info.grid_form[:n]),
            "grid_step": list(info.grid_step[:n]), "graph_builds": info.graph_builds,
            "autocorr_pending": list(info.autocorr_pending[:n]), "autocorr_fold_limit": info.autocorr_fold_limit,
            "grid_blocks": list(info.grid_blocks[:n])}


def epic_debug_schedule(plan: Plan, sub: int, n_time: int):
    """Owner workgroup and slot of every spectrum of sub-array ``sub`` in an
    accumulate call of ``n_time`` spectra: two int32 arrays [C * KS][n_time]."""
    if not 0 <= int(sub) < len(plan.subs) or int(n_time) < 1:   # let the library reject it
        _check(_lib.epic_debug_schedule(plan, int(sub), int(n_time), None, None), "epic_debug_schedule")
    info = epic_plan_query(plan)
    V = plan.subs[sub].n_chan * info["col_split"][sub]
    wg = np.empty((V, int(n_time)), dtype=np.int32)
    slot = np.empty_like(wg)
    _check(_lib.epic_debug_schedule(plan, int(sub), int(n_time), wg.ctypes.data_as(_P(ctypes.c_int32)),
                                    slot.ctypes.data_as(_P(ctypes.c_int32))), "epic_debug_schedule")
    return wg, slot


def epic_debug_geometry(plan: Plan, sub: int) -> np.ndarray:
    s = plan.subs[sub]
    out = np.zeros((int(s.n_chan), int(np.asarray(s.ant_xy).shape[0]), 2), dtype=np.int32)
    _check(_lib.epic_debug_geometry(plan, int(sub), out.ctypes.data_as(_P(ctypes.c_int32))), "epic_debug_geometry")
    return out


def epic_debug_unpack(d_bytes, n: int, nibble_order: int, d_out, stream=None):
    _check(_lib.epic_debug_unpack(_dev_ptr(d_bytes), int(n), int(nibble_order), _dev_ptr(d_out),
                                  _stream_handle(stream)), "epic_debug_unpack")


def epic_destroy(plan: Plan):
    if plan is None or plan.handle is None:
        return
    _check(_lib.epic_destroy(plan), "epic_destroy")
    plan.handle = None


class Imager:
    """Convenience owner of a plan and its output cubes (torch, on ``device``)."""

    def __init__(self, subs: Sequence, precision="fp32", max_time: int = 1, device: int = 0, **kw):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.plan = epic_plan(subs, precision=precision, max_time=max_time, device=device, **kw)
        info = epic_plan_query(self.plan)
        self.info = info
        self.images: List = [torch.empty((int(s.n_chan), info["npp"][k], int(s.grid_n), int(s.grid_n)),
                                         dtype=torch.float32, device=self.device) for k, s in enumerate(subs)]

    def accumulate(self, samples: Sequence, n_time: Optional[int] = None, stream=None):
        if n_time is None:
            n_time = int(samples[0].shape[0])
        epic_grid_fft_accumulate(self.plan, samples, n_time, stream)

    def readout(self, reset: bool = True, stream=None):
        epic_readout(self.plan, self.images, 1 if reset else 0, stream)
        return self.images

    def close(self):
        if self.plan is not None:
            epic_destroy(self.plan)
            self.plan = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False
