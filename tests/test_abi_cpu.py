"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before any side effect, and its FP64
geometry is bit-identical to the oracle's (dry-run plans touch no device)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epic.h")


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:epic_status|const char\*|int32_t)\s+(epic_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_entry_points():
    fns = declared_functions()
    for f in ("epic_plan", "epic_grid_fft_accumulate", "epic_readout", "epic_destroy", "epic_status_str"):
        assert f in fns


def test_library_exports_every_declared_symbol(E):
    lib = ctypes.CDLL(E.library_path())
    for f in declared_functions():
        assert hasattr(lib, f), f
    assert set(declared_functions()) == set(E.EXPORTED)
    assert E.epic_abi_version() == 1


def test_status_strings(E):
    names = ["EPIC_OK", "EPIC_E_ARG", "EPIC_E_GEOMETRY", "EPIC_E_NOMEM", "EPIC_E_DEVICE", "EPIC_E_UNSUPPORTED",
             "EPIC_E_STATE"]
    for k, n in enumerate(names):
        assert E.epic_status_str(k) == n
    assert E.epic_status_str(99) == "EPIC_E_UNKNOWN"


def dry(E, subs, **kw):
    kw.setdefault("max_time", 1000)
    return E.epic_plan(subs, flags=E.EPIC_F_DRY_RUN | kw.pop("flags", 0), **kw)


@pytest.mark.parametrize("cfg", [1, 2, 4, 5])
def test_geometry_bit_exact_with_oracle(E, cfg):
    wl = synth.workload(cfg)
    p = dry(E, wl.subs)
    for k, s in enumerate(wl.subs):
        cells = E.epic_debug_geometry(p, k)
        ref, _ = oracle.geometry(s)
        assert np.array_equal(cells, ref)
    E.epic_destroy(p)


def test_geometry_ties_round_up(E):
    class S:  # lambda = 1 m, dl = 0.5: x = 0.25 m is exactly half a cell
        ant_xy = np.array([[0.25, -0.25], [0.75, 0.0], [0.0, 0.0]])
        n_pol, n_chan, grid_n, grid_dl, freq0_hz, dfreq_hz, kernel_k = 1, 1, 32, 0.5, 299792458.0, 0.0, 3
    p = dry(E, [S()])
    assert E.epic_debug_geometry(p, 0)[0].tolist() == [[17, 16], [18, 16], [16, 16]]
    E.epic_destroy(p)


def test_dry_run_query(E):
    wl = synth.workload(2)
    p = dry(E, wl.subs)
    info = E.epic_plan_query(p)
    assert info["n_sub"] == 1 and info["npp"] == [4]
    assert info["slots"][0] >= 1 and info["threads"][0] == 512   # 8 lanes per column x 64 columns
    assert 16 <= info["window_max"][0] <= 24   # ~16 lambda aperture + 3-tap kernel, padded to 8
    assert info["lds_bytes"][0] <= 160 * 1024
    E.epic_destroy(p)


def test_dry_run_refuses_device_work(E):
    p = dry(E, synth.workload(1).subs)
    with pytest.raises(E.EpicError) as e:
        E.epic_grid_fft_accumulate(p, [1 << 20], 1, stream=0)
    assert e.value.status == E.EPIC_E_STATE
    with pytest.raises(E.EpicError) as e:
        E.epic_readout(p, [1 << 20], 0, stream=0)
    assert e.value.status == E.EPIC_E_STATE
    E.epic_destroy(p)


def test_stale_handle_rejected(E):
    p = dry(E, synth.workload(1).subs)
    h = p.handle
    E.epic_destroy(p)
    p.handle = h                     # use after destroy
    with pytest.raises(E.EpicError) as e:
        E.epic_plan_query(p)
    assert e.value.status == E.EPIC_E_ARG
    p.handle = None


class Sub:
    def __init__(self, **kw):
        self.ant_xy = np.array([[0.0, 0.0], [3.0, -2.0]])
        self.n_pol, self.n_chan, self.grid_n, self.grid_dl = 2, 2, 32, 0.5
        self.freq0_hz, self.dfreq_hz, self.kernel_k = 40e6, 25e3, 3
        self.__dict__.update(kw)


@pytest.mark.parametrize("bad,code", [
    (dict(n_pol=3), "ARG"), (dict(n_chan=0), "ARG"), (dict(grid_n=40), "ARG"), (dict(grid_n=272), "ARG"),
    (dict(kernel_k=2), "ARG"), (dict(kernel_k=9), "ARG"), (dict(grid_dl=0.0), "ARG"), (dict(grid_dl=np.nan), "ARG"),
    (dict(freq0_hz=-1.0), "ARG"), (dict(dfreq_hz=-1.0), "ARG"),
    (dict(ant_xy=np.array([[0.0, np.inf]])), "ARG"),
    (dict(ant_xy=np.array([[60.0, 0.0]])), "GEOMETRY"),          # 60 m at 40 MHz, dl 0.5 -> cell 32 of 32
    (dict(ant_xy=np.zeros((40000, 2))), "ARG"),                    # A * P > 65536
])
def test_validation(E, bad, code):
    with pytest.raises(E.EpicError) as e:
        dry(E, [Sub(**bad)])
    assert e.value.status == getattr(E, "EPIC_E_" + code)


def test_plan_level_validation(E):
    s = [Sub()]
    for kw, code in [(dict(max_time=0), "ARG"), (dict(precision=7), "ARG"), (dict(gridder=9), "ARG"),
                     (dict(output=5), "ARG"), (dict(reserved=(0, 1, 0, 0)), "ARG"), (dict(flags=1 << 20), "ARG"),
                     (dict(device=-1), "ARG")]:
        with pytest.raises(E.EpicError) as e:
            dry(E, s, **kw)
        assert e.value.status == getattr(E, "EPIC_E_" + code), kw
    with pytest.raises(E.EpicError):
        dry(E, [])
    # Stokes output needs two polarisations
    with pytest.raises(E.EpicError) as e:
        dry(E, [Sub(n_pol=1)], output=E.EPIC_OUT_STOKES)
    assert e.value.status == E.EPIC_E_ARG


def test_geometry_at_the_edge_is_accepted(E):
    # footprint exactly touching cells 0 and N-1
    lam = 299792458.0 / 40e6
    xy = np.array([[-15 * 0.5 * lam, 0.0], [14 * 0.5 * lam, 0.0]])
    p = dry(E, [Sub(ant_xy=xy, n_chan=1, dfreq_hz=0.0)])
    cells = E.epic_debug_geometry(p, 0)
    assert cells[0, :, 0].tolist() == [1, 30]
    E.epic_destroy(p)


def test_debug_calls_validate(E):
    with pytest.raises(E.EpicError) as e:
        E.epic_debug_unpack(0, 16, 0, 0, stream=0)
    assert e.value.status == E.EPIC_E_ARG
    with pytest.raises(E.EpicError) as e:
        E.epic_debug_unpack(1 << 20, -1, 0, 1 << 20, stream=0)
    assert e.value.status == E.EPIC_E_ARG


class _FakeTensor:
    """Stands in for a device tensor: the binding checks dtype and size
    before any pointer reaches the library."""

    def __init__(self, dtype, n):
        self.dtype, self._n, self.is_cuda = dtype, n, True

    def numel(self):
        return self._n

    def is_contiguous(self):
        return True

    def data_ptr(self):
        return 0x1000


def test_binding_checks_buffers_before_the_library(E):
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=16)
    plan = E.epic_plan([sub], max_time=4, flags=E.EPIC_F_DRY_RUN)
    try:
        need = 4 * 2 * 16 * 2
        for bad, msg in ((_FakeTensor("torch.uint8", need - 1), "elements needed"),
                         (_FakeTensor("torch.float32", need), "uint8 tensor expected")):
            with pytest.raises(ValueError, match=msg):
                E.epic_grid_fft_accumulate(plan, [bad], 4, stream=0)
        with pytest.raises(ValueError, match="one sample buffer per sub-array"):
            E.epic_grid_fft_accumulate(plan, [], 4, stream=0)
        with pytest.raises(ValueError, match="elements needed"):
            E.epic_readout(plan, [_FakeTensor("torch.float32", 2 * 4 * 64 * 64 - 1)], 1, stream=0)
        with pytest.raises(ValueError, match="float32 tensor expected"):
            E.epic_efield(plan, 0, _FakeTensor("torch.uint8", need), 4,
                          _FakeTensor("torch.float16", 4 * 2 * 2 * 64 * 64 * 2), stream=0)
        with pytest.raises(ValueError, match="gains"):
            E.epic_set_gains(plan, 0, np.ones((2, 16, 2, 1), dtype=np.float32), stream=0)
        # right sizes reach the library, which refuses a dry-run plan
        with pytest.raises(E.EpicError) as ei:
            E.epic_grid_fft_accumulate(plan, [_FakeTensor("torch.uint8", need)], 4, stream=0)
        assert ei.value.status == E.EPIC_E_STATE
    finally:
        E.epic_destroy(plan)


def test_plans_from_several_threads(E):
    """Separate plans may be created, queried and destroyed from different
    host threads at once (the library keeps its table of live plans under a
    lock)."""
    import threading
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=32)
    errors, done = [], []

    def work():
        try:
            for _ in range(15):
                plan = E.epic_plan([sub], max_time=4, flags=E.EPIC_F_DRY_RUN)
                assert E.epic_plan_query(plan)["n_sub"] == 1
                E.epic_destroy(plan)
                done.append(1)
        except Exception as exc:   # reported by the main thread
            errors.append(exc)

    threads = [threading.Thread(target=work) for _ in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors[0]
    assert len(done) == 8 * 15


def test_autocorr_fold_limit_setting(E, monkeypatch):
    """The zero-lag sums fold before 2^24 - 1 spectra (int32-exact: every
    term is at most 128); EPIC_AUTOCORR_FOLD_LIMIT lowers it, and values
    outside [1, 2^24 - 1] or not a number keep the default."""
    s = [Sub()]
    for env, want in ((None, (1 << 24) - 1), ("7", 7), ("0", (1 << 24) - 1), ("abc", (1 << 24) - 1),
                      (str(1 << 25), (1 << 24) - 1)):
        if env is None:
            monkeypatch.delenv("EPIC_AUTOCORR_FOLD_LIMIT", raising=False)
        else:
            monkeypatch.setenv("EPIC_AUTOCORR_FOLD_LIMIT", env)
        p = dry(E, s, flags=E.EPIC_F_REMOVE_AUTOCORR)
        try:
            info = E.epic_plan_query(p)
            assert info["autocorr_fold_limit"] == want, env
            assert info["autocorr_pending"] == [0]
        finally:
            E.epic_destroy(p)


def test_binding_refuses_to_load_without_the_library(tmp_path):
    """The product path has no CPU fallback: a copy of the package without
    libepic.so fails on import, naming the missing library."""
    import shutil
    import subprocess
    import sys as _sys
    pkg = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2301_09662_amd")
    dst = tmp_path / "paper_2301_09662_amd"
    dst.mkdir()
    for f in ("__init__.py", "epic.py"):
        shutil.copy(os.path.join(pkg, f), dst / f)
    r = subprocess.run([_sys.executable, "-c", "import paper_2301_09662_amd.epic"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "libepic.so is missing" in r.stderr and "no CPU fallback" in r.stderr
