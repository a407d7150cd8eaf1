"""Partial-accumulator slots across calls: the first accumulate call after a
reset (or after planning) stores its sums into the zeroed slots, every later
call of the same integration adds to them.  Integrations of several calls,
read out with and without reset, eager and replayed from captured graphs
(one graph per call length, inputs and first-call-or-not), against the
oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_parity, torch_dev


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def _subs(which):
    if which == "station":
        return [synth.shrink(synth.workload(2).subs[0], n_chan=3)]
    if which == "uneven":
        return [synth.shrink(s, n_chan=n) for s, n in zip(synth.workload(4).subs, (2, 1, 1))]
    return [synth.workload(1).subs[0]]   # 16 antennas, single pol


CASES = [("station", "fp32", "gather", 0), ("station", "fp32", "gather", "graph"),
         ("station", "fp16", "gather", "graph"), ("station", "fp16", "block", 0),
         ("station", "fp8", "block", "graph"), ("tiny", "fp16", "direct", "graph"),
         ("uneven", "fp16", "gather", "graph+one"), ("uneven", "fp16", "gather", 0)]


@pytest.mark.gpu
@pytest.mark.parametrize("which,precision,gridder,mode", CASES)
def test_first_call_stores_later_calls_add(E, which, precision, gridder, mode):
    torch, dev = torch_dev()
    subs = _subs(which)
    n = 5
    xs = [synth.samples(s, 2 * n) for s in subs]
    d = [torch.from_numpy(x).to(dev) for x in xs]
    half = [oracle.image(s, x[:n]) for s, x in zip(subs, xs)]
    full = [oracle.image(s, x) for s, x in zip(subs, xs)]
    flags = {0: 0, "graph": E.EPIC_F_GRAPH, "graph+one": E.EPIC_F_GRAPH | E.EPIC_F_ONE_LAUNCH}[mode]
    tol = 1e-5 if precision == "fp32" else 1e-3
    plan = E.epic_plan(subs, precision=precision, gridder=gridder, max_time=n, flags=flags)
    try:
        info = E.epic_plan_query(plan)

        def out():
            return [torch.full((s.n_chan, info["npp"][k], s.grid_n, s.grid_n), float("nan"), device=dev)
                    for k, s in enumerate(subs)]

        def acc(t0):
            E.epic_grid_fft_accumulate(plan, [x[t0:t0 + n] for x in d], n)

        def check(o, ref, what):
            torch.cuda.synchronize()
            for k in range(len(subs)):
                assert_parity(o[k].double().cpu().numpy(), ref[k], tol, f"{what} sub {k}")

        for rep in range(2):                        # two whole integrations of two calls each
            acc(0)
            acc(n)
            o = out()
            E.epic_readout(plan, o, 1)
            check(o, full, f"integration {rep}")
        acc(0)                                      # read out halfway without reset, then go on
        o = out()
        E.epic_readout(plan, o, 0)
        check(o, half, "halfway")
        acc(n)
        o = out()
        E.epic_readout(plan, o, 1)
        check(o, full, "after the halfway read-out")
        acc(n)                                      # the two halves the other way round
        acc(0)
        o = out()
        E.epic_readout(plan, o, 1)
        check(o, full, "reversed halves")
        if flags & E.EPIC_F_GRAPH:
            # each input buffer captured once as a first call and once as an
            # adding call
            assert E.epic_plan_query(plan)["graph_builds"] == 4
    finally:
        E.epic_destroy(plan)


@pytest.mark.gpu
def test_three_buffers_two_call_integrations_replay(E):
    """A caller rotating over three input buffers with integrations of two
    calls: six (buffer, first-call-or-not) graphs, captured in the first
    round and replayed in the second, every integration equal to the oracle."""
    torch, dev = torch_dev()
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2)
    n = 4
    x = synth.samples(sub, 3 * n)
    d = torch.from_numpy(x).to(dev)
    bufs = [d[k * n:(k + 1) * n] for k in range(3)]
    plan = E.epic_plan([sub], precision="fp32", max_time=n, flags=E.EPIC_F_GRAPH)
    try:
        for rnd in range(2):
            for a, b in ((0, 1), (2, 0), (1, 2)):
                E.epic_grid_fft_accumulate(plan, [bufs[a]], n)
                E.epic_grid_fft_accumulate(plan, [bufs[b]], n)
                o = torch.full((2, 4, 64, 64), float("nan"), device=dev)
                E.epic_readout(plan, [o], 1)
                torch.cuda.synchronize()
                ref = oracle.image(sub, np.concatenate([x[a * n:(a + 1) * n], x[b * n:(b + 1) * n]]))
                assert_parity(o.double().cpu().numpy(), ref, 1e-5, f"round {rnd} buffers {a}, {b}")
            assert E.epic_plan_query(plan)["graph_builds"] == 6
    finally:
        E.epic_destroy(plan)
