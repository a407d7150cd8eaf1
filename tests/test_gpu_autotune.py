"""The plan-time autotuner: per sub-array it times the gather form (gather
program in LDS or streamed) against the block-GEMM form at every step size
that fits, keeps the fastest, and with EPIC_TUNE_CACHE stores the choice
(keyed by device architecture and plan shape) for later plans to reuse
untimed.  Whatever it picks must give the oracle's image."""
import json

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_parity, run_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def test_tuned_plan_from_timing_then_from_cache(E, tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("EPIC_TUNE_CACHE", str(cache))
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=4)
    x = synth.samples(sub, 24)
    ora = oracle.image(sub, x)
    (g1,), i1 = run_library(E, [sub], [x], precision="fp16", flags=E.EPIC_F_AUTOTUNE)
    assert i1["autotuned"] == 1
    assert_parity(g1, ora, 1e-3, "tuned by timing")
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    key, val = next(iter(entries.items()))
    assert "gfx" in key and val.startswith(f"g{i1['grid_form'][0]},tb{i1['grid_step'][0]}")
    (g2,), i2 = run_library(E, [sub], [x], precision="fp16", flags=E.EPIC_F_AUTOTUNE)
    assert i2["autotuned"] == 2
    assert (i2["grid_form"], i2["grid_step"], i2["lds_bytes"]) == (i1["grid_form"], i1["grid_step"], i1["lds_bytes"])
    assert np.array_equal(g1, g2)


def test_cache_entries_naming_no_candidate_are_timed_again(E, tmp_path, monkeypatch):
    """A cache entry whose choice is not a candidate of the plan (a stale or
    edited file) is ignored: the plan times its candidates and rewrites it."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("EPIC_TUNE_CACHE", str(cache))
    sub = synth.shrink(synth.workload(4).subs[1], n_chan=3)
    x = synth.samples(sub, 10)
    (_,), i1 = run_library(E, [sub], [x], precision="fp16", flags=E.EPIC_F_AUTOTUNE)
    entries = json.loads(cache.read_text())
    key = next(iter(entries))
    cache.write_text(json.dumps({key: "g9,tb7,prog3|0|1"}))
    (g,), i2 = run_library(E, [sub], [x], precision="fp16", flags=E.EPIC_F_AUTOTUNE)
    assert i2["autotuned"] == 1
    assert json.loads(cache.read_text())[key] != "g9,tb7,prog3|0|1"
    assert_parity(g, oracle.image(sub, x), 1e-3, "re-tuned")


def test_uneven_batch_tuned_and_cached(E, tmp_path, monkeypatch):
    """Three uneven sub-arrays: each one's form, then the single launch against
    one launch each, timed once and then reused from the cache."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("EPIC_TUNE_CACHE", str(cache))
    wl = synth.workload(4)
    subs = [synth.shrink(s, n_chan=n) for s, n in zip(wl.subs, (3, 2, 2))]
    xs = [synth.samples(s, 12) for s in subs]
    gs, i1 = run_library(E, subs, xs, precision="fp16", flags=E.EPIC_F_AUTOTUNE)
    assert i1["autotuned"] == 1
    gs2, i2 = run_library(E, subs, xs, precision="fp16", flags=E.EPIC_F_AUTOTUNE)
    assert i2["autotuned"] == 2
    assert (i2["batched"], i2["weight"], i2["grid_form"]) == (i1["batched"], i1["weight"], i1["grid_form"])
    for s, x, g, g2 in zip(subs, xs, gs, gs2):
        assert_parity(g, oracle.image(s, x), 1e-3, f"batch tuned N={s.grid_n}")
        assert np.array_equal(g, g2)
