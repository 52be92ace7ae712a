"""GPU checks of the jerk search (fdas_make_templates_jerk): one plane per w.

The GPU integrates A(q, z, w) by Gauss-Legendre quadrature, the oracle by the
Simpson rule (different methods; both ~1e-9).  Bars: FP64 bank within 1e-9
of the largest template value; FP32 planes within 1e-4 max(P64, 1) of the
oracle plane built from the oracle's jerk taps; BF16 (matrix-core) planes
within the BF16 bars of the plain path; an injected jerk chirp peaks at its
(z, r) cell on its own w plane with its matched power, and a scan over w
puts the maximum on the true w.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import plane as OP
from oracle import response as R

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def plan(dev, **kw):
    from paper_2206_12205_amd.fdas import Plan
    return Plan(device=dev, **kw)


@pytest.mark.parametrize("w", [24.0, -70.0])
def test_jerk_bank_matches_oracle(dev, w):
    import torch
    say(f"[jerk] bank w={w}")
    zs = R.z_grid(-8.0, 4.0, 5)
    pl = plan(dev, max_bins=8192, z_min=-8.0, z_step=4.0, n_z=5, n_taps=64, seg_len=1024, compute="fp64",
              plane_dtype="fp64")
    pl.make_templates(w=w)
    torch.cuda.synchronize()
    b = pl.bank().cpu().numpy()
    got = b[..., 0] + 1j * b[..., 1]
    want = R.template_spectra(zs, 64, 1024, w=w)
    assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want))
    # w = 0 through the jerk entry is the closed-form bank
    pl.make_templates(w=0.0)
    torch.cuda.synchronize()
    b0 = pl.bank().cpu().numpy()
    want0 = R.template_spectra(zs, 64, 1024)
    assert np.max(np.abs(b0[..., 0] + 1j * b0[..., 1] - want0)) <= 1e-12 * np.max(np.abs(want0))


@pytest.mark.parametrize("compute,algo", [("fp32", "valu"), ("bf16", "mfma")])
def test_jerk_plane_matches_oracle(dev, compute, algo):
    import torch
    say(f"[jerk] plane {compute}")
    n_t, M, w = 1 << 15, 64, 40.0
    x = synth.complex_chirp_spectrum(n_t, 5000.3, 6.0, amp=0.08, w=w)
    x = x + synth.random_spectrum(x.size, seed=9)
    zs = R.z_grid(-12.0, 3.0, 9)
    ref = OP.plane(x, R.template_taps(zs, M, w=w))
    pl = plan(dev, max_bins=x.size, z_min=-12.0, z_step=3.0, n_z=9, n_taps=M,
              seg_len=1024 if compute == "fp32" else 4096, compute=compute, algo=algo)
    pl.make_templates(w=w)
    p = pl.correlate(torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to(dev))
    p = p.double().cpu().numpy()
    err = np.abs(p - ref) / np.maximum(ref, 1.0)
    if compute == "fp32":
        assert err.max() <= 1e-4, f"{err.max():.2e}"
    else:
        bright = ref > 20.0
        assert err.max() <= 0.15 and err.mean() <= 0.02, f"{err.max():.3f} {err.mean():.4f}"
        assert np.max(np.abs(p[bright] - ref[bright]) / ref[bright]) <= 0.03
    assert np.unravel_index(np.argmax(p), p.shape) == np.unravel_index(np.argmax(ref), ref.shape)


def test_jerk_chirp_found_on_its_own_w_plane(dev):
    import torch
    say("[jerk] w scan")
    n_t, r_bar, z, w, M = 1 << 16, 12000, 8.0, 48.0, 128
    x = synth.complex_chirp_spectrum(n_t, r_bar - z / 2 - w / 6, z, amp=0.05, w=w)
    xd = torch.from_numpy(x).to(dev)
    pl = plan(dev, max_bins=x.size, z_min=-20.0, z_step=2.0, n_z=21, n_taps=M, compute="fp32")
    best = []
    for wt in (w - 24.0, w - 12.0, w, w + 12.0, w + 24.0):
        pl.make_templates(w=wt)
        p = pl.correlate(xd).double().cpu().numpy()
        j, r = np.unravel_index(np.argmax(p), p.shape)
        best.append((p[j, r], wt, j, r))
    pmax, wbest, j, r = max(best)
    assert wbest == w and (-20.0 + 2.0 * j, r) == (z, r_bar)
    e_ret = R.retained_energy([z], M, w=w)[0]
    assert abs(pmax / (0.05 ** 2 * n_t * e_ret) - 1.0) < 1e-3
