"""GPU spectrum preparation (fdas_prepare) against the oracle (oracle/prep.py).

Bars.  The GPU transform is single precision (the paper's real FFT), the
oracle's double: log2(N) radix passes each add a relative rounding of a few
2^-24 to every value, so a normalised spectrum (values of order one) agrees
within 2e-5 per bin at every size here; the median is an exact selection of
single-precision powers, so the GPU's normalised noise powers have median
ln 2 to single-precision rounding.  Downstream, the plane of the GPU-prepared
spectrum finds the same harmonic-band peaks as the plane of the oracle's.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import prep as OPR

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_prepare(x, dev):
    import torch
    from paper_2206_12205_amd.fdas import prepare
    return prepare(torch.from_numpy(np.asarray(x, dtype=np.float32)).to(dev)).cpu().numpy()


# the global-pass lengths (4 .. 32 samples, 2^25), the four-step form's
# smallest (64 = 8 x 4 complex, 384 = 24 x 8 with the radix-3 pass) and
# largest (2^24, 3 * 2^22) lengths, and 3 * 2^k lengths between
@pytest.mark.parametrize("n_t", [4, 8, 32, 64, 384, 1536, 2048, 4096, 6144, 1 << 17, 3 << 17, 1 << 20,
                                 3 << 20, 3 << 22, 1 << 24, 1 << 25])
def test_prepare_matches_oracle(dev, n_t):
    say(f"[prep] n_t={n_t}")
    rng = np.random.default_rng(n_t)
    x = (rng.normal(size=n_t) * 3.0 + 0.5).astype(np.float32)
    got = gpu_prepare(x, dev)
    want = OPR.prepare(x.astype(np.float64))
    assert got.shape == want.shape and got[0] == 0
    err = np.abs(got - want)
    assert err.max() <= 2e-5 * max(1.0, np.abs(want).max() / 10), f"{err.max():.2e}"
    if n_t >= 2048:
        p = np.sort(np.abs(got[1:].astype(np.complex128)) ** 2)
        assert abs(p[(p.size - 1) // 2] / math.log(2.0) - 1.0) < 2e-6


@pytest.mark.parametrize("n_t", [1 << 16, 3 << 16])
def test_prepare_degenerate_median(dev, n_t):
    """A unit impulse at t = 0: every bin k >= 1 has power exactly 1, so the
    median's histogram bin gathers every key of the spectrum and the exact
    selection runs over all of them; the result is sqrt(ln 2) in every bin."""
    x = np.zeros(n_t, dtype=np.float32)
    x[0] = 1.0
    got = gpu_prepare(x, dev)
    want = OPR.prepare(x.astype(np.float64))
    assert got[0] == 0 and np.allclose(want[1:], math.sqrt(math.log(2.0)))
    assert np.max(np.abs(got[1:] - want[1:])) <= 1e-6


def test_prepare_single_dm_series_then_plane(dev):
    """Full single-DM series (2^23 samples, trial 6: a bright pulsar): the GPU
    spectrum against the oracle's, then the BF16 plane of each: the same cell
    for the highest point of every harmonic band."""
    import torch
    from paper_2206_12205_amd import metrics
    from paper_2206_12205_amd.fdas import Plan, prepare
    c = synth.CONFIGS[2]
    say("[prep] single-DM series")
    x, p = synth.config2_series(6)                          # a bright pulsar (P1 ~ 3000)
    xs = torch.from_numpy(x.astype(np.float32)).to(dev)
    got = prepare(xs)
    want = OPR.prepare(x.astype(np.float32).astype(np.float64))
    err = np.abs(got.cpu().numpy() - want)
    assert err.max() <= 2e-5 * max(1.0, np.abs(want).max() / 10), f"{err.max():.2e}"
    n = got.numel()
    pl = Plan(max_bins=n, z_min=c["z_min"], z_step=c["z_step"], n_z=c["n_z"], n_taps=c["n_taps"],
              compute="bf16", plane_dtype="bf16", device=dev)
    pg = pl.correlate(got).float()
    po = pl.correlate(torch.from_numpy(want.astype(np.complex64)).to(dev)).float()
    T = c["n_t"] * c["tsamp"]
    bands = metrics.harmonic_bands(p.f, T, n, 8)
    mg, mo = metrics.band_maxima(pg, bands), metrics.band_maxima(po, bands)
    bright = [i for i, m in enumerate(mo) if m[2] > c["threshold"]]
    assert bright, "the workload's pulsar has bright harmonics"
    for i in bright:
        assert mg[i][:2] == mo[i][:2], f"band {i}"
        assert abs(mg[i][2] / mo[i][2] - 1.0) < 0.02
