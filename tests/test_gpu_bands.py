"""GPU band maxima (fdas_band_max) against the oracle's band_max: exact
selection (same cell, same value) on planes with many ties and NaN cells,
windows clipped at the edges, empty and all-NaN windows, windows wider than
one work chunk, and the harmonic bands of a full single-DM BF16 plane."""
import sys

import numpy as np
import pytest

import synth
from oracle import peaks as OPK

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def plan(dev, **kw):
    from paper_2206_12205_amd.fdas import Plan
    return Plan(device=dev, **kw)


def compare(got, want, what):
    z, r, p = want
    assert np.array_equal(got["z_idx"], z), what
    assert np.array_equal(got["r"], r), what
    pw = p.astype(np.float32)
    both_nan = np.isnan(pw) & np.isnan(got["power"])
    assert np.all(both_nan | (got["power"] == pw)), what


@pytest.mark.parametrize("pd", ["fp32", "bf16", "fp64"])
def test_band_max_ties_nan_clipping(dev, pd):
    import torch
    say(f"[bands] {pd}")
    n_z, n = 11, 20000
    rng = np.random.default_rng(3)
    Ph = np.round(rng.uniform(0, 6, size=(n_z, n)) * 4) / 4      # exact in bf16: many ties
    Ph[2, 100:9000] = np.nan
    Ph[5:7, 15000:15010] = np.nan
    Ph[9, 19990:] = 7.75                                         # a unique top value near the edge
    tdt = {"fp32": torch.float32, "bf16": torch.bfloat16, "fp64": torch.float64}[pd]
    P = torch.from_numpy(Ph).to(tdt).to(dev)
    windows = [(0, n_z, 0, n), (2, 3, 100, 9000), (2, 3, 50, 9100), (-4, 3, -10, 40), (9, 40, 19980, 30000),
               (5, 7, 15000, 15010), (3, 3, 0, 10), (0, 11, 4000, 13000), (1, 2, 7, 8), (6, 11, 0, 20000)]
    compute = "fp64" if pd == "fp64" else "fp32"
    pl = plan(dev, max_bins=n, z_min=-10.0, z_step=2.0, n_z=n_z, n_taps=16, compute=compute, plane_dtype=pd)
    got = pl.band_max(P, windows)
    want = OPK.band_max(P.to(torch.float64).cpu().numpy(), windows)
    compare(got, want, pd)


def test_band_max_single_dm_harmonic_bands(dev):
    """Table 3 bands of trial 0's pulsar on the full single-DM BF16 plane."""
    import torch
    from paper_2206_12205_amd import metrics
    c = synth.CONFIGS[2]
    say("[bands] single-DM bf16 harmonic bands")
    x, sp = synth.config2_device(dev, 0)
    n = x.numel()
    pl = plan(dev, max_bins=n, z_min=c["z_min"], z_step=c["z_step"], n_z=c["n_z"], n_taps=c["n_taps"],
              compute="bf16", plane_dtype="bf16")
    P = pl.correlate(x)
    bands = metrics.harmonic_bands(sp.pulsars[0].f, sp.T, n, 8)
    windows = [(0, c["n_z"], lo, hi) for lo, hi in bands if lo < hi]
    got = pl.band_max(P, windows)
    Ph = P.view(torch.int16).cpu().numpy().view(np.uint16)
    Pf = (Ph.astype(np.uint32) << 16).view(np.float32)
    want = OPK.band_max(Pf, windows)
    compare(got, want, "single-DM bands")
