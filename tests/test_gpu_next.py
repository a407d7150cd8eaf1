"""GPU parity of the steps adjacent to the hot path: autocorrelation removal
(every antenna's own a = b term subtracted at read-out), per-antenna complex
gains folded into the taps (changed between calls), and the Stokes output.

Tolerances as for the plain path (1e-5 FP32, 1e-3 FP16 per image), with the
errors of an autocorrelation-removed image measured against the norm and
peak of the full image: the GPU forms the full sum and the a = b image in
FP32 and subtracts, so its rounding scales with the full image, not with the
(smaller) difference.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_parity, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_2301_09662_amd import epic
    return epic


def removed_errors(gpu, ref, full):
    """Per-image errors of an autocorrelation-removed cube, normalised by the
    full image (cross products by sqrt(|XX| |YY|) of the full image)."""
    C, npp = ref.shape[:2]
    fro = np.zeros((C, npp))
    mx = np.zeros((C, npp))
    for c in range(C):
        nx = np.linalg.norm(full[c, 0])
        ny = np.linalg.norm(full[c, 1]) if npp == 4 else nx
        peak = np.abs(full[c, : min(npp, 2)]).max()
        for k in range(npp):
            den = np.linalg.norm(full[c, k]) if k < 2 else np.sqrt(nx * ny)
            fro[c, k] = np.linalg.norm(gpu[c, k] - ref[c, k]) / den
            mx[c, k] = np.abs(gpu[c, k] - ref[c, k]).max() / peak
    return fro.max(), mx.max()


def run_plan(E, subs, steps, precision="fp32", flags=0, output=0, taps=None, max_time=None):
    """steps: list of ("acc", [samples per sub]) / ("gains", sub, array or None) /
    ("read", reset); returns the list of read-out cubes (float64)."""
    torch, dev = torch_dev()
    mt = max_time or max(s[1][0].shape[0] for s in steps if s[0] == "acc")
    plan = E.epic_plan(subs, precision=precision, max_time=mt, flags=flags, output=output, taps=taps)
    outs = []
    try:
        info = E.epic_plan_query(plan)
        for st in steps:
            if st[0] == "acc":
                d = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in st[1]]
                E.epic_grid_fft_accumulate(plan, d, st[1][0].shape[0])
                torch.cuda.synchronize()
            elif st[0] == "gains":
                E.epic_set_gains(plan, st[1], st[2])
            else:
                o = [torch.full((s.n_chan, info["npp"][k], s.grid_n, s.grid_n), float("nan"), device=dev)
                     for k, s in enumerate(subs)]
                E.epic_readout(plan, o, st[1])
                torch.cuda.synchronize()
                outs.append([t.double().cpu().numpy() for t in o])
    finally:
        E.epic_destroy(plan)
    return outs


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 1e-3)])
def test_autocorr_removed_station_subset(E, precision, tol):
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=3)
    x = synth.samples(sub, 24)
    (out,) = run_plan(E, [sub], [("acc", [x]), ("read", 1)], precision, flags=E.EPIC_F_REMOVE_AUTOCORR)
    full = oracle.image(sub, x)
    ref = full - oracle.autocorr(sub, x)
    fro, mx = removed_errors(out[0], ref, full)
    print(f"{precision} autocorr removed: rel err {fro:.2e}, max |d|/peak {mx:.2e}; "
          f"removed / full image norm {np.linalg.norm(ref[:, 0]) / np.linalg.norm(full[:, 0]):.3f}")
    assert fro <= tol and mx <= tol


def test_autocorr_removed_single_pol_and_integrations(E):
    """Single pol, two integrations: the second read-out holds only its own
    spectra (accumulators and autocorrelations reset), split over two calls."""
    sub = synth.workload(1).subs[0]
    x = synth.samples(sub, 64)
    outs = run_plan(E, [sub], [("acc", [x[:40]]), ("read", 1), ("acc", [x[40:50]]), ("acc", [x[50:]]),
                               ("read", 1)], flags=E.EPIC_F_REMOVE_AUTOCORR, max_time=40)
    for o, xs in zip(outs, (x[:40], x[40:])):
        full = oracle.image(sub, xs)
        fro, mx = removed_errors(o[0], full - oracle.autocorr(sub, xs), full)
        assert fro <= 1e-5 and mx <= 1e-5


def test_autocorr_removed_batched_graph(E):
    subs = [synth.shrink(s, n_chan=n) for s, n in zip(synth.workload(4).subs, (2, 2, 1))]
    xs = [synth.samples(s, 12) for s in subs]
    flags = E.EPIC_F_REMOVE_AUTOCORR | E.EPIC_F_GRAPH | E.EPIC_F_AUTOTUNE
    (out,) = run_plan(E, subs, [("acc", [x[:6] for x in xs]), ("acc", [x[6:] for x in xs]), ("read", 1)],
                      "fp16", flags=flags)
    for k, (s, x) in enumerate(zip(subs, xs)):
        full = oracle.image(s, x)
        fro, mx = removed_errors(out[k], full - oracle.autocorr(s, x), full)
        assert fro <= 1e-3 and mx <= 1e-3, f"sub {k}: {fro:.2e} {mx:.2e}"


def test_autocorr_removed_user_complex_taps(E):
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=64)
    x = synth.samples(sub, 16)
    taps = np.random.default_rng(11).standard_normal((2, 64, 2, 3, 3, 2)).astype(np.float32)
    (out,) = run_plan(E, [sub], [("acc", [x]), ("read", 1)], flags=E.EPIC_F_REMOVE_AUTOCORR, taps=[taps])
    full = oracle.image(sub, x, taps=taps)
    fro, mx = removed_errors(out[0], full - oracle.autocorr(sub, x, taps=taps), full)
    assert fro <= 1e-5 and mx <= 1e-5


def user_taps(z):
    """complex [C][A][P][K][K] -> float32 [C][A][P][K][K][2] (the taps argument)."""
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).astype(np.float32))


def gained_taps(sub, taps, gains):
    """Taps (float32 [...][2]) times per-antenna gains, product in FP64: what
    the library folds into its gather weights before rounding to FP32."""
    t = taps[..., 0].astype(np.float64) + 1j * taps[..., 1]
    g = gains[..., 0].astype(np.float64) + 1j * gains[..., 1]
    return user_taps(t * g[:, :, :, None, None])


def test_gains_between_calls_with_autocorr_removal(E):
    """Complex gains g1 for the first call, g2 for the second, within one
    integration: the image is the sum of the two calls' images with their own
    gains, and the removed a = b terms follow the gains of each call."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=96)
    x = synth.samples(sub, 20)
    rng = np.random.default_rng(12)
    taps = user_taps(oracle.taps(sub))                              # the default Gaussian, as user taps
    g1 = rng.standard_normal((2, 96, 2, 2)).astype(np.float32)
    g2 = rng.standard_normal((2, 96, 2, 2)).astype(np.float32)
    flags = E.EPIC_F_REMOVE_AUTOCORR | E.EPIC_F_COMPLEX_WEIGHTS
    steps = [("gains", 0, g1), ("acc", [x[:8]]), ("gains", 0, g2), ("acc", [x[8:]]), ("read", 1)]
    (out,) = run_plan(E, [sub], steps, flags=flags, taps=[taps])
    t1, t2 = gained_taps(sub, taps, g1), gained_taps(sub, taps, g2)
    full = oracle.image(sub, x[:8], taps=t1) + oracle.image(sub, x[8:], taps=t2)
    ref = full - oracle.autocorr(sub, x[:8], taps=t1) - oracle.autocorr(sub, x[8:], taps=t2)
    fro, mx = removed_errors(out[0], ref, full)
    assert fro <= 1e-5 and mx <= 1e-5


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 1e-3)])
def test_gains_complex_and_reset_to_unit(E, precision, tol):
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=128)
    x = synth.samples(sub, 10)
    g = np.random.default_rng(13).standard_normal((2, 128, 2, 2)).astype(np.float32)
    steps = [("gains", 0, g), ("acc", [x]), ("read", 1), ("gains", 0, None), ("acc", [x]), ("read", 1)]
    o1, o2 = run_plan(E, [sub], steps, precision, flags=E.EPIC_F_COMPLEX_WEIGHTS)
    taps = user_taps(oracle.taps(sub))
    assert_parity(o1[0], oracle.image(sub, x, taps=gained_taps(sub, taps, g)), tol, "gains")
    assert_parity(o2[0], oracle.image(sub, x), tol, "unit gains again")


def test_real_gains_and_refusals(E):
    """Real-weight plans take real gains: equal X and Y gains where one weight
    serves both pols (the default kernel), per-pol gains where the taps differ
    per pol; complex gains, or unequal ones on shared weights, are refused."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=1, n_ant=64)
    x = synth.samples(sub, 6)
    rng = np.random.default_rng(14)
    g = np.zeros((1, 64, 2, 2), dtype=np.float32)
    g[..., 0, 0] = rng.uniform(0.5, 2.0, (1, 64))
    g[..., 1, 0] = g[..., 0, 0]                                   # equal per pol
    (o,) = run_plan(E, [sub], [("gains", 0, g), ("acc", [x]), ("read", 1)])
    taps = user_taps(oracle.taps(sub))
    assert_parity(o[0], oracle.image(sub, x, taps=gained_taps(sub, taps, g)), 1e-5, "shared weights, real gains")
    # per-pol real taps: per-pol real gains
    t2 = taps.copy()
    t2[:, :, 1, ..., 0] *= 0.75                                   # Y taps differ from X
    g2 = g.copy()
    g2[..., 1, 0] = rng.uniform(0.5, 2.0, (1, 64))
    (o2,) = run_plan(E, [sub], [("gains", 0, g2), ("acc", [x]), ("read", 1)], taps=[t2])
    assert_parity(o2[0], oracle.image(sub, x, taps=gained_taps(sub, t2, g2)), 1e-5, "per-pol weights, real gains")
    plan = E.epic_plan([sub], max_time=6)
    try:
        for bad in (g2, np.where(np.arange(2) == 1, 0.5, g)):   # unequal per pol; a complex part
            with pytest.raises(E.EpicError) as ei:
                E.epic_set_gains(plan, 0, np.ascontiguousarray(bad, dtype=np.float32))
            assert ei.value.status == E.EPIC_E_UNSUPPORTED
        gn = g.copy()
        gn[0, 1, 1, 0] = np.nan
        with pytest.raises(E.EpicError) as ei:
            E.epic_set_gains(plan, 0, gn)
        assert ei.value.status == E.EPIC_E_ARG
    finally:
        E.epic_destroy(plan)


@pytest.mark.parametrize("flags", [0, 8])
def test_stokes_output(E, flags):
    """I = XX+YY, Q = XX-YY, U = 2 Re XY*, V = 2 Im XY* (linear feeds), also
    after autocorrelation removal."""
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2)
    x = synth.samples(sub, 12)
    (o,) = run_plan(E, [sub], [("acc", [x]), ("read", 1)], flags=flags, output=E.EPIC_OUT_STOKES)
    full = oracle.image(sub, x)
    pol = full - (oracle.autocorr(sub, x) if flags else 0.0)
    st = np.stack([pol[:, 0] + pol[:, 1], pol[:, 0] - pol[:, 1], 2 * pol[:, 2], 2 * pol[:, 3]], axis=1)
    fst = np.stack([full[:, 0] + full[:, 1], full[:, 0] - full[:, 1], 2 * full[:, 2], 2 * full[:, 3]], axis=1)
    peak = np.abs(fst[:, 0]).max()
    assert np.abs(o[0] - st).max() <= 1e-5 * peak


@pytest.mark.parametrize("cfg,k,nchan,nant,T,wide", [(1, 0, 4, None, 6, 0), (2, 0, 3, None, 5, 0),
                                                     (4, 1, 2, None, 4, 0), (5, 0, 1, 512, 2, 0),
                                                     (2, 0, 1, None, 2, 256)])
def test_efield_images(E, cfg, k, nchan, nant, T, wide):
    """Per-spectrum field images of each polarisation against the oracle's,
    phases included (N = 32 single pol, 64, 48, and 128 with the column
    split), to 1e-5 per image."""
    torch, dev = torch_dev()
    sub = synth.shrink(synth.workload(cfg).subs[k], n_chan=nchan, n_ant=nant)
    if wide:
        import dataclasses
        sub = dataclasses.replace(sub, grid_n=wide, grid_dl=0.5)
    x = synth.samples(sub, T)
    ora = oracle.efield(sub, x)                                   # [T][C][P][N][N]
    plan = E.epic_plan([sub], max_time=T)
    try:
        out = torch.full((T, sub.n_chan, sub.n_pol, sub.grid_n, sub.grid_n, 2), float("nan"), device=dev)
        E.epic_efield(plan, 0, torch.from_numpy(x).to(dev), T, out)
        torch.cuda.synchronize()
        g = out.double().cpu().numpy()
    finally:
        E.epic_destroy(plan)
    g = g[..., 0] + 1j * g[..., 1]
    assert np.isfinite(g).all()
    err = np.linalg.norm(g - ora, axis=(-2, -1)) / np.linalg.norm(ora, axis=(-2, -1))
    print(f"efield cfg{cfg}: max per-image rel err {err.max():.2e}")
    assert err.max() <= 1e-5


def test_efield_refused_for_fp16(E):
    torch, dev = torch_dev()
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=1)
    plan = E.epic_plan([sub], precision="fp16", max_time=2)
    try:
        x = torch.zeros((2, 1, sub.n_ant, 2), dtype=torch.uint8, device=dev)
        out = torch.zeros((2, 1, 2, 64, 64, 2), device=dev)
        with pytest.raises(E.EpicError) as ei:
            E.epic_efield(plan, 0, x, 2, out)
        assert ei.value.status == E.EPIC_E_UNSUPPORTED
    finally:
        E.epic_destroy(plan)


def test_gains_changed_between_graph_replays(E):
    """A graph replays the captured kernels; gains set between replays reach
    it through the rebuilt gather weights (same buffers)."""
    torch, dev = torch_dev()
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2, n_ant=64)
    x = synth.samples(sub, 8)
    d = torch.from_numpy(x).to(dev)
    rng = np.random.default_rng(31)
    taps = user_taps(oracle.taps(sub))
    plan = E.epic_plan([sub], max_time=8, flags=E.EPIC_F_GRAPH | E.EPIC_F_COMPLEX_WEIGHTS)
    try:
        for r in range(3):
            g = rng.standard_normal((2, 64, 2, 2)).astype(np.float32)
            E.epic_set_gains(plan, 0, g)
            E.epic_grid_fft_accumulate(plan, [d], 8)
            o = torch.zeros((2, 4, 64, 64), device=dev)
            E.epic_readout(plan, [o], 1)
            torch.cuda.synchronize()
            assert_parity(o.double().cpu().numpy(), oracle.image(sub, x, taps=gained_taps(sub, taps, g)), 1e-5,
                          f"graph replay {r} with new gains")
    finally:
        E.epic_destroy(plan)


def test_two_plans_on_two_streams(E):
    """Two plans enqueued on two streams at once give the same images as
    run one after the other."""
    torch, dev = torch_dev()
    a = synth.shrink(synth.workload(2).subs[0], n_chan=3)
    b = synth.shrink(synth.workload(4).subs[1], n_chan=4)
    xa, xb = synth.samples(a, 20), synth.samples(b, 20)
    da, db = torch.from_numpy(xa).to(dev), torch.from_numpy(xb).to(dev)
    pa = E.epic_plan([a], max_time=20)
    pb = E.epic_plan([b], precision="fp16", max_time=20)
    try:
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        oa = torch.zeros((3, 4, 64, 64), device=dev)
        ob = torch.zeros((4, 4, 48, 48), device=dev)
        torch.cuda.synchronize()
        for _ in range(3):
            E.epic_grid_fft_accumulate(pa, [da], 20, sa)
            E.epic_grid_fft_accumulate(pb, [db], 20, sb)
        E.epic_readout(pa, [oa], 1, sa)
        E.epic_readout(pb, [ob], 1, sb)
        torch.cuda.synchronize()
        ref_a = 3 * oracle.image(a, xa)
        ref_b = 3 * oracle.image(b, xb)
        assert_parity(oa.double().cpu().numpy(), ref_a, 1e-5, "stream a")
        assert_parity(ob.double().cpu().numpy(), ref_b, 1e-3, "stream b")
    finally:
        E.epic_destroy(pa)
        E.epic_destroy(pb)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 1e-3)])
def test_autocorr_removed_and_stokes_on_split_columns(E, precision, tol):
    """Autocorrelation removal and the Stokes output on a 128 grid whose image
    columns span two workgroups (512 antennas of the large array)."""
    sub = synth.shrink(synth.workload(5).subs[0], n_chan=2, n_ant=512)
    x = synth.samples(sub, 6)
    (o,) = run_plan(E, [sub], [("acc", [x]), ("read", 1)], precision, flags=E.EPIC_F_REMOVE_AUTOCORR,
                    output=E.EPIC_OUT_STOKES)
    full = oracle.image(sub, x)
    pol = full - oracle.autocorr(sub, x)
    st = np.stack([pol[:, 0] + pol[:, 1], pol[:, 0] - pol[:, 1], 2 * pol[:, 2], 2 * pol[:, 3]], axis=1)
    fst = np.stack([full[:, 0] + full[:, 1], full[:, 0] - full[:, 1], 2 * full[:, 2], 2 * full[:, 3]], axis=1)
    peak = np.abs(fst[:, 0]).max()
    assert np.abs(o[0] - st).max() <= tol * peak


@pytest.mark.parametrize("sign", [-1, 1])
def test_stokes_v_sign_of_a_circular_source(E, sign):
    """The sign of V is fixed by the voltages: a noise-free point source whose
    Y field is E_Y = sign * i * E_X gives XY* = -sign i |E_X|^2, so
    V = 2 Im XY* = -sign * I at its pixel (and Q = U = 0 there): V = +I for
    E_Y = -i E_X.  The samples are exact 4-bit integers (amplitude 5)."""
    torch, dev = torch_dev()
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=1)
    N = sub.grid_n
    i0, j0 = N // 2 + 7, N // 2 - 5
    l0, m0 = sub.pixel_lm(i0, j0)
    lam = 299792458.0 / sub.freq0_hz
    u, v = sub.ant_xy[:, 0] / lam, sub.ant_xy[:, 1] / lam
    rng = np.random.default_rng(40)
    T = 6
    s = rng.choice([1, -1, 1j, -1j], size=T)                          # source signal per spectrum
    ph = np.exp(-2j * np.pi * (u * l0 + v * m0))                      # plane-wave phase, Eq. 1
    ex = np.round((5 * s[:, None] * ph[None, :]).real) + 1j * np.round((5 * s[:, None] * ph[None, :]).imag)
    ey = sign * 1j * ex                                               # exact: swaps and negates components
    x = np.zeros((T, 1, sub.n_ant, 2), dtype=np.uint8)
    x[:, 0, :, 0] = synth.pack44(ex.real, ex.imag)
    x[:, 0, :, 1] = synth.pack44(ey.real, ey.imag)
    (o,) = run_plan(E, [sub], [("acc", [x]), ("read", 1)], output=E.EPIC_OUT_STOKES)
    I, Q, U, V = o[0][0]
    assert np.unravel_index(np.argmax(I), I.shape) == (j0, i0)
    assert abs(V[j0, i0] + sign * I[j0, i0]) <= 1e-5 * I[j0, i0]
    assert abs(Q[j0, i0]) <= 1e-5 * I[j0, i0] and abs(U[j0, i0]) <= 1e-5 * I[j0, i0]


def test_autocorr_folds_before_the_exact_range_ends(E, monkeypatch):
    """With the fold count lowered to 7 spectra, calls of 5 fold the pending
    zero-lag sums before adding to them once they would pass 7; the image is
    unchanged (folding only moves exact sums into the lag accumulator)."""
    monkeypatch.setenv("EPIC_AUTOCORR_FOLD_LIMIT", "7")
    torch, dev = torch_dev()
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2)
    x = synth.samples(sub, 15)
    plan = E.epic_plan([sub], max_time=5, flags=E.EPIC_F_REMOVE_AUTOCORR)
    try:
        info = E.epic_plan_query(plan)
        assert info["autocorr_fold_limit"] == 7
        d = torch.from_numpy(x).to(dev)
        pend = []
        for k in range(3):
            E.epic_grid_fft_accumulate(plan, [d[5 * k:5 * k + 5]], 5)
            pend.append(E.epic_plan_query(plan)["autocorr_pending"][0])
        assert pend == [5, 5, 5]
        out = torch.empty((2, 4, 64, 64), device=dev)
        E.epic_readout(plan, [out], 1)
        assert E.epic_plan_query(plan)["autocorr_pending"][0] == 0
        torch.cuda.synchronize()
        full = oracle.image(sub, x)
        ref = full - oracle.autocorr(sub, x)
        fro, mx = removed_errors(out.double().cpu().numpy(), ref, full)
        assert fro <= 1e-5 and mx <= 1e-5
    finally:
        E.epic_destroy(plan)


def test_graph_cache_alternating_buffers(E):
    """A caller rotating over two input buffers replays two captured graphs
    instead of capturing on every call; every replay is right."""
    torch, dev = torch_dev()
    sub = synth.shrink(synth.workload(2).subs[0], n_chan=2)
    x = synth.samples(sub, 12)
    bufs = [torch.from_numpy(x[:6].copy()).to(dev), torch.from_numpy(x[6:].copy()).to(dev)]
    ref = [oracle.image(sub, x[:6]), oracle.image(sub, x[6:])]
    plan = E.epic_plan([sub], max_time=6, flags=E.EPIC_F_GRAPH)
    try:
        out = torch.empty((2, 4, 64, 64), device=dev)
        for k in range(6):
            E.epic_grid_fft_accumulate(plan, [bufs[k % 2]], 6)
            E.epic_readout(plan, [out], 1)
            torch.cuda.synchronize()
            assert_parity(out.double().cpu().numpy(), ref[k % 2], 1e-5, f"graph replay {k}")
        assert E.epic_plan_query(plan)["graph_builds"] == 2
    finally:
        E.epic_destroy(plan)
