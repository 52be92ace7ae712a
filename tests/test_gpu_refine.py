"""GPU parity of candidate refinement (fdas_refine / fdas_refine_backward)
against the FP64 oracle (oracle/refine.py: responses by the Fresnel closed
form, derivatives by Gauss-Legendre quadrature of the differentiated
integrand — a different method from the kernel's integration by parts)."""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import refine as ORF

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def chirps_spectrum(n_t=1 << 14, seed=0):
    """Noise plus three complex chirps (integer and fractional r, several z)."""
    g = np.random.default_rng(seed)
    x = (g.standard_normal(n_t // 2) + 1j * g.standard_normal(n_t // 2)) / math.sqrt(2.0)
    for r_bar, z, amp in ((1500.3, 8.6, 0.2), (3000.0, -25.0, 0.3), (5000.7, 0.2, 0.15)):
        x += synth.complex_chirp_spectrum(n_t, r_bar - z / 2, z, amp).astype(np.complex128)
    return x.astype(np.complex64)


def test_refine_values_and_gradients_match_oracle(dev):
    import torch
    from paper_2206_12205_amd.fdas import refine
    say("[refine] oracle values")
    x = chirps_spectrum()
    g = np.random.default_rng(1)
    r = np.concatenate([[1500.25, 3000.6, 5000.9, 10.4, 8180.5], g.uniform(20, 8000, 31)])
    z = np.concatenate([[8.0, -24.0, 0.0, 3.0, 0.3], g.uniform(-40, 40, 31)])
    z[7] = 0.0
    z[8] = 1e-7
    z[9] = -0.49
    # both sides of the switch from quadrature to the closed form (|z| = 0.05)
    z[10], z[11], z[12], z[13] = 0.0501, -0.0499, 0.049, -0.06
    xs = torch.from_numpy(x).to(dev)
    _, _, P, gr, gz = refine(xs, torch.from_numpy(r), torch.from_numpy(z))
    P, gr, gz = (t.cpu().numpy() for t in (P, gr, gz))
    Po, gro, gzo = ORF.power_grad(x, r, z)
    scale = np.maximum(Po, 1.0)
    assert np.max(np.abs(P - Po) / scale) < 1e-9
    assert np.max(np.abs(gr - gro) / scale) < 1e-8
    assert np.max(np.abs(gz - gzo) / scale) < 1e-8


@pytest.mark.parametrize("taps", [2, 16, 32, 34, 64])
def test_refine_tap_counts_and_odd_batches(dev, taps):
    """Two candidates share a wave up to 32 taps (a 32-lane segment each),
    one takes the whole wave above: values and gradients match the oracle for
    every tap count, with an odd number of candidates (the last wave holds
    one) and candidates at both ends of the spectrum."""
    import torch
    from paper_2206_12205_amd.fdas import refine
    say(f"[refine] {taps} taps, 31 candidates")
    x = chirps_spectrum()
    g = np.random.default_rng(taps)
    r = np.concatenate([[1500.25, 0.3, x.size - 1.6], g.uniform(20, 8000, 28)])
    z = np.concatenate([[8.0, 2.0, -3.0], g.uniform(-40, 40, 28)])
    _, _, P, gr, gz = refine(torch.from_numpy(x).to(dev), torch.from_numpy(r), torch.from_numpy(z), taps=taps)
    P, gr, gz = (t.cpu().numpy() for t in (P, gr, gz))
    Po, gro, gzo = ORF.power_grad(x, r, z, taps)
    scale = np.maximum(Po, 1.0)
    assert np.max(np.abs(P - Po) / scale) < 1e-9
    assert np.max(np.abs(gr - gro) / scale) < 1e-8
    assert np.max(np.abs(gz - gzo) / scale) < 1e-8


def test_refine_gradient_matches_finite_differences(dev):
    import torch
    from paper_2206_12205_amd.fdas import refine
    say("[refine] finite differences")
    x = torch.from_numpy(chirps_spectrum(seed=2)).to(dev)
    g = np.random.default_rng(3)
    r = g.uniform(50, 8000, 40)
    r = np.floor(r) + np.clip(r - np.floor(r), 0.05, 0.95)       # keep r +- h inside one window
    z = g.uniform(-30, 30, 40)
    # central differences: truncation error h^2 |d3P| / 6 (1.5e-5 relative at
    # h = 1e-3) and rounding error ~1e-12 P / h; h = 2e-4 keeps both < 1e-6
    h = 2e-4
    T = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64))
    _, _, P, gr, gz = refine(x, T(r), T(z))
    Prp = refine(x, T(r + h), T(z))[2]
    Prm = refine(x, T(r - h), T(z))[2]
    Pzp = refine(x, T(r), T(z + h))[2]
    Pzm = refine(x, T(r), T(z - h))[2]
    fr = ((Prp - Prm) / (2 * h)).cpu().numpy()
    fz = ((Pzp - Pzm) / (2 * h)).cpu().numpy()
    scale = np.maximum(P.cpu().numpy(), 1.0)
    assert np.max(np.abs(gr.cpu().numpy() - fr) / scale) < 1e-5
    assert np.max(np.abs(gz.cpu().numpy() - fz) / scale) < 1e-5


def test_refine_ascent_matches_oracle(dev):
    import torch
    from paper_2206_12205_amd.fdas import refine
    say("[refine] 20-step ascent")
    x = chirps_spectrum(seed=4)
    r0 = np.array([1500.0, 1499.8, 3000.4, 2999.6, 5000.5, 5001.1, 1500.9, 3000.0])
    z0 = np.array([8.0, 9.5, -24.0, -26.0, 0.0, 1.0, 7.2, -25.5])
    xs = torch.from_numpy(x).to(dev)
    r, z, P, gr, gz = (t.cpu().numpy() for t in refine(xs, torch.from_numpy(r0), torch.from_numpy(z0),
                                                         n_steps=20))
    ro, zo, Po, gro, gzo = ORF.ascend(x, r0, z0, steps=20)
    assert np.max(np.abs(r - ro)) < 1e-7
    assert np.max(np.abs(z - zo)) < 1e-6
    assert np.max(np.abs(P - Po) / np.maximum(Po, 1.0)) < 1e-9
    # converged near the injected chirps
    assert abs(r[0] - 1500.3) < 0.02 and abs(z[0] - 8.6) < 0.1


def test_autograd_function(dev):
    import torch
    from paper_2206_12205_amd.fdas import interpolated_power, refine
    say("[refine] autograd")
    x = torch.from_numpy(chirps_spectrum(seed=5)).to(dev)
    r = torch.tensor([1500.2, 3000.3, 4000.7], dtype=torch.float64, device=dev, requires_grad=True)
    z = torch.tensor([8.0, -25.0, 3.3], dtype=torch.float64, device=dev, requires_grad=True)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=dev)
    loss = (interpolated_power(r, z, x) * w).sum()
    loss.backward()
    _, _, P, gr, gz = refine(x, r.detach(), z.detach())
    assert torch.allclose(r.grad, w * gr, rtol=1e-12, atol=0)
    assert torch.allclose(z.grad, w * gz, rtol=1e-12, atol=0)
    rr = r.detach().clone().requires_grad_(True)
    zz = z.detach().clone().requires_grad_(True)
    # eps balances the FP64 noise of P (~1e-12 relative, divided by eps) and
    # the truncation error eps^2 |d3P| / 6 (P ~ 1500 at these chirps)
    assert torch.autograd.gradcheck(lambda a, b: interpolated_power(a, b, x), (rr, zz), eps=5e-5, atol=1e-3,
                                    rtol=1e-5)


def test_refine_single_dm_candidates(dev):
    """The single-DM flow: candidates at the 4096 highest local maxima of the
    FP32 plane plus seeded offsets U[-0.5, 0.5] x U[-1, 1], 32 taps, 20
    ascent steps; a sample checked against the oracle's ascent."""
    import torch
    from paper_2206_12205_amd.fdas import Plan, refine
    c = synth.CONFIGS[2]
    say("[refine] single-DM candidates")
    sp = synth.config2(0)
    n = sp.spec.size
    x = torch.from_numpy(sp.spec).to(dev)
    pl = Plan(n, c["z_min"], c["z_step"], c["n_z"], c["n_taps"], c["seg_len"], compute="fp32", device=dev)
    plane = pl.correlate(x)
    pk = pl.peaks(plane, 8.0, capacity=1 << 20)
    assert pk["n_found"] >= 4096
    top = np.argsort(-pk["power"], kind="stable")[:4096]
    dr, dz = synth.refine_offsets(4096)
    r0 = pk["r"][top].astype(np.float64) + dr
    z0 = c["z_min"] + c["z_step"] * pk["z_idx"][top].astype(np.float64) + dz
    r, z, P, gr, gz = refine(x, torch.from_numpy(r0), torch.from_numpy(z0), n_steps=20)
    P0 = refine(x, torch.from_numpy(r0), torch.from_numpy(z0))[2]
    r, z, P, P0 = (t.cpu().numpy() for t in (r, z, P, P0))
    assert np.mean(P >= P0 * (1 - 1e-9)) > 0.95        # ascent does not lose power
    idx = np.linspace(0, 4095, 12).astype(int)
    ro, zo, Po, _, _ = ORF.ascend(sp.spec, r0[idx], z0[idx], steps=20)
    assert np.max(np.abs(r[idx] - ro)) < 1e-6
    assert np.max(np.abs(z[idx] - zo)) < 1e-5
    assert np.max(np.abs(P[idx] - Po) / np.maximum(Po, 1.0)) < 1e-8
