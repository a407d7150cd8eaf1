"""The work split of the persistent launches, checked on the host through
epic_debug_schedule (the same split and slot functions the kernels run):
every spectrum has exactly one owner workgroup, a workgroup's spectra of one
virtual channel are contiguous in time, its slot is inside the plan's slot
count, and two workgroups never add into the same slot of one channel (the
partial sums need no atomics).  Covers one-sub-array FP32 and FP16 plans and
the batched FP16 plan of sub-arrays of unequal cost, including calls so short
that one spectrum costs more than a workgroup's share."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def check_split(E, plan, sub, n_time):
    info = E.epic_plan_query(plan)
    wg, slot = E.epic_debug_schedule(plan, sub, n_time)
    S = info["slots"][sub]
    assert (wg >= 0).all() and (wg < info["workgroups"][sub]).all()
    assert (slot >= 0).all() and (slot < S).all()
    for v in range(wg.shape[0]):
        owners, first = np.unique(wg[v], return_index=True)
        # contiguous pieces: the owner changes exactly len(owners) - 1 times
        assert np.count_nonzero(np.diff(wg[v])) == len(owners) - 1
        # one slot per owner, distinct across owners
        s_of = slot[v][first]
        assert len(np.unique(s_of)) == len(owners)
        for o, s in zip(owners, s_of):
            assert (slot[v][wg[v] == o] == s).all()
    return wg, slot


def dry(E, subs, precision, max_time, flags=0):
    return E.epic_plan(subs, precision=precision, max_time=max_time, flags=E.EPIC_F_DRY_RUN | flags)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
@pytest.mark.parametrize("n_time", [1, 2, 7, 999, 1000])
def test_station_split(E, precision, n_time):
    p = dry(E, synth.workload(2).subs, precision, 1000)
    try:
        check_split(E, p, 0, n_time)
    finally:
        E.epic_destroy(p)


@pytest.mark.parametrize("one_launch", [True, False])
@pytest.mark.parametrize("n_time", [1, 2, 3, 5, 17, 250])
def test_uneven_batch_split(E, n_time, one_launch):
    """Both forms of a plan of sub-arrays: one persistent launch for all of
    them (cost-weighted split) and one dedicated launch each."""
    wl = synth.workload(4)
    p = dry(E, wl.subs, "fp16", wl.n_time, flags=E.EPIC_F_ONE_LAUNCH if one_launch else 0)
    try:
        info = E.epic_plan_query(p)
        assert info["can_batch"] == 1 and info["batched"] == (1 if one_launch else 0)
        assert min(info["weight"]) >= 1
        # the N=96 array has the most expensive spectra in the cost model
        assert info["weight"][2] == max(info["weight"])
        for k in range(3):
            check_split(E, p, k, n_time)
    finally:
        E.epic_destroy(p)


def test_heavy_spectra_get_one_owner_each(E):
    """A batch with one channel per sub-array and short calls: a spectrum
    costs more than a workgroup's share, so each has its own owner and the
    slot is the spectrum index, which must stay below the slot count even
    where max_time caps it."""
    subs = [synth.shrink(s, n_chan=1) for s in synth.workload(4).subs]
    p = dry(E, subs, "fp16", 3, flags=E.EPIC_F_ONE_LAUNCH)
    try:
        info = E.epic_plan_query(p)
        assert info["batched"] == 1 and max(info["slots"]) <= 3
        G = info["workgroups"][0]
        for n_time in (1, 2, 3):
            total = sum(s.n_chan * info["col_split"][k] * n_time * info["weight"][k] for k, s in enumerate(subs))
            Lc = -(-total // G)
            heavy = [k for k in range(3) if info["weight"][k] >= Lc]
            assert heavy, "no sub-array in the one-owner-per-spectrum regime"
            for k in range(3):
                wg, slot = check_split(E, p, k, n_time)
                if k in heavy:
                    assert len(np.unique(wg)) == wg.size
                    assert (slot == np.arange(n_time)[None, :]).all()
    finally:
        E.epic_destroy(p)


def test_one_launch_refused_where_it_cannot_run(E):
    a = synth.shrink(synth.workload(4).subs[1], n_chan=2)
    b = synth.shrink(synth.workload(1).subs[0], n_chan=2)        # single pol: another kernel family
    with pytest.raises(E.EpicError) as ei:
        dry(E, [a, b], "fp16", 4, flags=E.EPIC_F_ONE_LAUNCH)
    assert ei.value.status == E.EPIC_E_UNSUPPORTED
    with pytest.raises(E.EpicError):
        dry(E, [a], "fp32", 4, flags=E.EPIC_F_ONE_LAUNCH)


def test_schedule_validates(E):
    p = dry(E, synth.workload(1).subs, "fp32", 10)
    try:
        for bad in (0, 11, -1):
            with pytest.raises(E.EpicError):
                E.epic_debug_schedule(p, 0, bad)
        with pytest.raises(E.EpicError):
            E.epic_debug_schedule(p, 1, 5)
    finally:
        E.epic_destroy(p)


def wide_grid(sub, n, dl):
    """The same array imaged on an n x n grid of spacing dl wavelengths."""
    import dataclasses
    return dataclasses.replace(sub, grid_n=n, grid_dl=dl)


@pytest.mark.parametrize("n,dl,ks", [(256, 0.5, 8), (192, 0.5, 8)])
def test_wide_grid_split(E, n, dl, ks):
    """256 x 256 and 192 x 192 grids: each spectrum's columns span eight
    workgroups; the column-part-major split still gives every spectrum one
    owner per part and distinct slots."""
    sub = wide_grid(synth.shrink(synth.workload(2).subs[0], n_chan=6), n, dl)
    p = dry(E, [sub], "fp32", 40)
    try:
        info = E.epic_plan_query(p)
        assert info["col_split"][0] == ks
        for n_time in (1, 3, 40):
            check_split(E, p, 0, n_time)
    finally:
        E.epic_destroy(p)


def test_grid_sizes_without_a_kernel(E):
    base = synth.shrink(synth.workload(2).subs[0], n_chan=1)
    for n, prec in ((240, "fp32"), (224, "fp16"), (80, "fp16")):
        with pytest.raises(E.EpicError) as ei:
            dry(E, [wide_grid(base, n, 0.5)], prec, 4)
        assert ei.value.status == E.EPIC_E_UNSUPPORTED, (n, prec)
    with pytest.raises(E.EpicError) as ei:
        dry(E, [wide_grid(base, 272, 0.5)], "fp32", 4)
    assert ei.value.status == E.EPIC_E_ARG


def test_arrays_too_large_for_lds_are_refused(E):
    """20000 dual-pol antennas need more LDS for one spectrum's decoded
    samples than a workgroup has: the plan says so instead of launching."""
    import dataclasses
    base = synth.shrink(synth.workload(2).subs[0], n_chan=1)
    rng = np.random.default_rng(1)
    big = dataclasses.replace(base, ant_xy=rng.uniform(-40, 40, (20000, 2)))
    for prec in ("fp32", "fp16"):
        with pytest.raises(E.EpicError) as ei:
            dry(E, [big], prec, 4)
        assert ei.value.status == E.EPIC_E_UNSUPPORTED


def test_window_spanning_a_256_grid_is_refused(E):
    """Antennas whose footprints span the whole 256 x 256 grid: the window
    (and its 16-bit cell offsets) does not fit a workgroup, so the plan says
    so rather than launching."""
    import dataclasses
    base = synth.shrink(synth.workload(2).subs[0], n_chan=1)
    lam = 299792458.0 / base.freq0_hz
    d = 126 * base.grid_dl * lam
    xy = np.array([[-d, -d], [d, d], [-d, d], [d, -d]])
    sub = dataclasses.replace(base, ant_xy=xy, grid_n=256)
    for prec in ("fp32", "fp16"):
        with pytest.raises(E.EpicError) as ei:
            dry(E, [sub], prec, 4)
        assert ei.value.status == E.EPIC_E_UNSUPPORTED
