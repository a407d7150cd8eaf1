"""Host-side pieces of bench.py: the NumPy FP32 CPU context baseline computes
the same images as the oracle, and the executed-MFMA model counts the
station's 176 matrix-core products per channel and spectrum."""
import numpy as np

import bench
import oracle
import synth


def test_numpy_baseline_matches_oracle():
    for cfg, nch in ((1, None), (2, 2)):
        sub = synth.workload(cfg).subs[0]
        if nch:
            sub = synth.shrink(sub, n_chan=nch)
        x = synth.samples(sub, 12)
        ora = oracle.image(sub, x)
        for c in range(sub.n_chan):
            img = bench.numpy_fft_image(sub, x[:, c], c)
            assert np.abs(img - ora[c]).max() <= 1e-5 * np.abs(ora[c]).max()


def test_mfma_model_station():
    from paper_2301_09662_amd import epic as E
    subs = synth.workload(2).subs
    plan = E.epic_plan(subs, precision="fp16", max_time=4, flags=E.EPIC_F_DRY_RUN)
    try:
        assert bench.mfma_ops_per_spectrum(plan, subs) == 176 * subs[0].n_chan
    finally:
        E.epic_destroy(plan)
