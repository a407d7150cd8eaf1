"""The allocation-free entry point epic_image_noalloc against the existing
accumulate + read-out entry points, through the C ABI.

Each case runs two calls in a row, the second with fewer spectra, and checks
both images against epic_grid_fft_accumulate + epic_readout(reset) of the same
plan on the same input.  Both routes run the same kernels on the same
spectra; only the order in which the partial accumulators are summed can
differ, so the bar is the FP32 path's 1e-5 per image for every precision.
"""

import numpy as np
import pytest

import synth
from gpu_util import assert_parity, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def _reference(E, plan, subs, xs, n, dev, torch):
    """accumulate + readout(reset) of the first n spectra."""
    info = E.epic_plan_query(plan)
    outs = [torch.full((s.n_chan, info["npp"][k], s.grid_n, s.grid_n), float("nan"), device=dev)
            for k, s in enumerate(subs)]
    E.epic_grid_fft_accumulate(plan, [x[:n] for x in xs], n)
    E.epic_readout(plan, outs, 1)
    return outs


def _noalloc(E, plan, subs, xs, n, dev, torch):
    info = E.epic_plan_query(plan)
    outs = [torch.full((s.n_chan, info["npp"][k], s.grid_n, s.grid_n), float("nan"), device=dev)
            for k, s in enumerate(subs)]
    E.epic_image_noalloc(plan, [x[:n] for x in xs], n, outs)
    return outs


def _check_two_calls(E, subs, T, T2, precision="fp32", flags=0):
    torch, dev = torch_dev()
    xs = [torch.from_numpy(synth.samples(s, T)).to(dev) for s in subs]
    plan = E.epic_plan(subs, precision=precision, max_time=T, flags=flags)
    try:
        for n in (T, T2):      # the second call is smaller and reuses the dirty scratch
            got = _noalloc(E, plan, subs, xs, n, dev, torch)
            ref = _reference(E, plan, subs, xs, n, dev, torch)
            torch.cuda.synchronize()
            for k, (g, r) in enumerate(zip(got, ref)):
                g, r = g.double().cpu().numpy(), r.double().cpu().numpy()
                assert np.isfinite(g).all()
                assert_parity(g, r, TOL, f"noalloc {precision} sub {k}, {n} spectra")
    finally:
        E.epic_destroy(plan)


def test_noalloc_fp32_station(E):
    _check_two_calls(E, [synth.shrink(synth.workload(2).subs[0], n_chan=6)], 40, 13)


def test_noalloc_fp16_uneven_batch(E):
    """A batched FP16 plan of two sub-arrays (one launch each here)."""
    subs = [synth.shrink(synth.workload(4).subs[0], n_chan=3), synth.shrink(synth.workload(4).subs[1], n_chan=4)]
    _check_two_calls(E, subs, 24, 5, precision="fp16", flags=E.EPIC_F_ONE_LAUNCH)


def test_noalloc_stokes_single_pol_and_zero_spectra(E):
    torch, dev = torch_dev()
    s1 = synth.shrink(synth.workload(1).subs[0], n_chan=2)
    _check_two_calls(E, [s1], 30, 1)
    s2 = synth.shrink(synth.workload(2).subs[0], n_chan=2)
    x = torch.from_numpy(synth.samples(s2, 4)).to(dev)
    plan = E.epic_plan([s2], max_time=4, output=E.EPIC_OUT_STOKES)
    try:
        out = torch.full((2, 4, 64, 64), float("nan"), device=dev)
        E.epic_image_noalloc(plan, [x], 4, [out])
        ref = _reference(E, plan, [s2], [x], 4, dev, torch)[0]
        torch.cuda.synchronize()
        assert_parity(out.double().cpu().numpy(), ref.double().cpu().numpy(), TOL, "noalloc stokes")
        E.epic_image_noalloc(plan, [x], 0, [out])                  # no spectra: zero images
        torch.cuda.synchronize()
        assert float(out.abs().max()) == 0.0
    finally:
        E.epic_destroy(plan)


def test_noalloc_size_limit_and_refusals(E):
    """A plan whose partial accumulators exceed the static buffer is refused
    for a long call and accepted for one spectrum (one slot per channel);
    autocorrelation removal and calls beyond max_time are refused."""
    torch, dev = torch_dev()
    wide = synth.shrink(synth.workload(6).subs[0], n_chan=40)
    per_slot = wide.n_chan * 4 * wide.grid_n ** 2 * 4
    assert per_slot < E.NOALLOC_MAX_BYTES < 2 * per_slot
    x = torch.from_numpy(synth.samples(wide, 4)).to(dev)
    plan = E.epic_plan([wide], max_time=4)
    try:
        assert E.epic_plan_query(plan)["slots"][0] >= 2
        out = torch.empty((40, 4, 256, 256), device=dev)
        with pytest.raises(E.EpicError) as e:
            E.epic_image_noalloc(plan, [x], 4, [out])
        assert e.value.status == E.EPIC_E_NOMEM
        x5 = torch.from_numpy(synth.samples(wide, 5)).to(dev)
        with pytest.raises(E.EpicError) as e:
            E.epic_image_noalloc(plan, [x5], 5, [out])    # beyond max_time
        assert e.value.status == E.EPIC_E_ARG
        E.epic_image_noalloc(plan, [x], 1, [out])
        ref = _reference(E, plan, [wide], [x], 1, dev, torch)[0]
        torch.cuda.synchronize()
        assert_parity(out.double().cpu().numpy(), ref.double().cpu().numpy(), TOL, "noalloc wide, 1 spectrum")
    finally:
        E.epic_destroy(plan)
    s = synth.shrink(synth.workload(2).subs[0], n_chan=2)
    plan = E.epic_plan([s], max_time=4, flags=E.EPIC_F_REMOVE_AUTOCORR)
    try:
        y = torch.from_numpy(synth.samples(s, 4)).to(dev)
        with pytest.raises(E.EpicError) as e:
            E.epic_image_noalloc(plan, [y], 4, [torch.empty((2, 4, 64, 64), device=dev)])
        assert e.value.status == E.EPIC_E_UNSUPPORTED
    finally:
        E.epic_destroy(plan)
