"""GPU check of the whole single-series search (pipeline.search_series):
preparation, the plane with its peaks and the harmonic sums with their
peaks, each one fused library call.  Each list must equal the step-by-step
calls on the same intermediate (fdas_correlate + fdas_peaks,
fdas_harmonic_sum + fdas_peaks), and the injected pulsar of the single-DM
series (trial 6, a bright one) must be found: a peak within 2 bins of its
fundamental's mean frequency in the plane and in every harmonic sum (which
gathers the harmonics onto the fundamental's cell)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_search_series_single_dm(dev):
    import torch
    from paper_2206_12205_amd.fdas import Plan
    from paper_2206_12205_amd.pipeline import search_series
    c = synth.CONFIGS[2]
    say("[search] single-DM series, trial 6")
    x, p = synth.config2_series(6)
    xs = torch.from_numpy(x.astype(np.float32)).to(dev)
    n = x.size // 2
    pl = Plan(max_bins=n, z_min=c["z_min"], z_step=c["z_step"], n_z=c["n_z"], n_taps=c["n_taps"],
              compute="bf16", plane_dtype="bf16", device=dev)
    thr = {1: c["threshold"], 2: c["threshold"] + 10.0, 4: c["threshold"] + 20.0, 8: c["threshold"] + 30.0}
    spec, plane, found = search_series(pl, xs, thr, harmonics=(1, 2, 4, 8))
    T = c["n_t"] * c["tsamp"]
    r1 = p.r_bar(T)
    # the same lists as the step-by-step calls on the same intermediates
    ref = pl.peaks(pl.correlate(spec), thr[1])
    assert ref["n_found"] == found[1]["n_found"] and np.array_equal(ref["r"], found[1]["r"])
    for h in (2, 4, 8):
        S = pl.harmonic_sum(plane, h)
        ref = pl.peaks(S, thr[h])
        assert ref["n_found"] == found[h]["n_found"], f"H={h}"
        assert np.array_equal(ref["r"], found[h]["r"]) and np.array_equal(ref["z_idx"], found[h]["z_idx"])
    # the pulsar: found at its fundamental in the plane and in every sum
    for h in (1, 2, 4, 8):
        r = found[h]["r"]
        assert found[h]["n_found"] > 0 and np.min(np.abs(r - r1)) <= 2, f"H={h}: nearest {np.min(np.abs(r - r1))}"
