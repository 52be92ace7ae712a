"""Pins of the oracle's acceleration response and templates.

The response is defined as A(q, z) = int_0^1 exp(i pi (2 q u + z u^2)) du (the
Fourier response of a linearly drifting sinusoid, Ransom et al. 2002, cited in
Section "Introduction"); the oracle evaluates it through Fresnel integrals.
These tests fix it against things other than that closed form.
"""
import math

import numpy as np
import pytest

from oracle import response as R


def simpson(q, z, n=400_000):
    """Composite Simpson rule on the defining integral (independent method)."""
    u = np.linspace(0.0, 1.0, n + 1)
    w = np.ones(n + 1)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    w /= 3.0 * n
    return np.sum(w * np.exp(1j * np.pi * (2 * q * u + z * u * u)))


CASES = [(0.3, 2.0), (5.2, 6.4), (-40.5, 100.0), (-3.3, 2.0), (10.0, 0.5),
         (-60.0, 100.0), (1.0, 1e-4), (0.0, 3.0), (-3.0, 3.0), (-1.5, 3.0),
         (128.7, 200.0), (-300.2, 200.0), (2.5, -7.0), (-50.0, -100.0),
         (7.25, 0.0), (0.0, 0.0), (0.7, 5e-4), (0.7, 2e-3), (30.0, -1e-5)]


@pytest.mark.parametrize("q,z", CASES)
def test_closed_form_matches_quadrature(q, z):
    a = complex(R.response(q, z))
    b = simpson(q, z)
    assert abs(a - b) <= 1e-9 * max(1.0, abs(b)) + 1e-11, (a, b)


def test_z_zero_is_fourier_interpolation_and_identity():
    # z = 0: A(q, 0) = exp(i pi q) sinc(q); at integer q it is the Kronecker delta
    m = np.arange(-40, 41, dtype=np.float64)
    a = R.response(m, 0.0)
    want = np.zeros_like(a)
    want[m == 0] = 1.0
    assert np.max(np.abs(a - want)) < 1e-15
    g = R.template_taps([0.0], 64)[0]
    assert abs(g[32] - 1.0) < 1e-15 and np.max(np.abs(np.delete(g, 32))) < 1e-15


def test_conjugate_symmetry():
    q = np.linspace(-50, 50, 37)
    for z in (2.0, 37.5, 180.0):
        assert np.max(np.abs(R.response(q, -z) - np.conj(R.response(-q, z)))) < 1e-12


@pytest.mark.parametrize("z,delta", [(0.0, 0.37), (6.4, 0.37), (100.0, 0.11), (-64.0, 0.5)])
def test_parseval(z, delta):
    # sum over all integer k of |A(r0 - k, z)|^2 = int_0^1 |e^{...}|^2 du = 1.
    # Truncated to |k - r_bar| <= K the tail decays like 1 / (pi^2 K).
    K = 4000
    r0 = 0.5 * (-z) + delta                  # mean frequency r_bar = delta
    k = np.arange(-K, K + 1, dtype=np.float64)
    s = np.sum(np.abs(R.response(r0 - k, z)) ** 2)
    assert s <= 1.0 + 1e-12
    assert 1.0 - s <= 3.0 / (math.pi ** 2 * K)
    if z == 0.0:
        # pure sinc^2: tail = 2 sin^2(pi delta) / (pi^2 K) to leading order
        pred = 1.0 - 2.0 * math.sin(math.pi * delta) ** 2 / (math.pi ** 2 * K)
        assert abs(s - pred) < 2e-7


def test_branch_continuity():
    # Y1 crosses zero at q = 0; the small-|z| quadrature meets the closed form
    for z in (3.0, 50.0):
        a = R.response(np.array([-1e-9, 1e-9]), z)
        assert abs(a[0] - a[1]) < 1e-8
        a = R.response(np.array([-z - 1e-9, -z + 1e-9]), z)
        assert abs(a[0] - a[1]) < 1e-8
    q = np.array([0.3, 4.0, -17.0])
    lo = R.response(q, 0.999e-3)
    hi = R.response(q, 1.001e-3)
    assert np.max(np.abs(lo - hi)) < 1e-5


def test_dft_of_sampled_chirp_approaches_response():
    # the DFT of a sampled unit chirp, divided by N, is a Riemann sum of A
    n = 1 << 14
    r0, z = 1000.3, 12.0
    u = np.arange(n) / n
    x = np.exp(2j * np.pi * (r0 * u + 0.5 * z * u * u))
    X = np.fft.fft(x) / n
    k = np.arange(980, 1030)
    a = R.response(r0 - k, z)
    assert np.max(np.abs(X[k] - a)) < 2e-4


def test_derivatives_match_finite_differences():
    q = np.array([0.3, -4.7, 12.2, -0.01])
    for z in (0.0, 2.0, -30.0, 90.0):
        dq, dz = R.response_grad(q, z)
        h = 1e-5
        fq = (R.response(q + h, z) - R.response(q - h, z)) / (2 * h)
        fz = (R.response(q, z + h) - R.response(q, z - h)) / (2 * h)
        if z == 0.0:   # the small-z branch is quadrature on both sides; use h>=1e-3 jump-free
            h = 1e-6
            fz = (R.response(q, z + h) - R.response(q, z - h)) / (2 * h)
        assert np.max(np.abs(dq - fq)) < 1e-7
        assert np.max(np.abs(dz - fz)) < 1e-6


def test_templates_unit_norm_and_symmetric_magnitude():
    zs = R.z_grid(-16.0, 2.0, 17)
    g = R.template_taps(zs, 64)
    assert np.max(np.abs(np.linalg.norm(g, axis=1) - 1.0)) < 1e-14
    # mean-frequency centring: |g_z[m]| equals |g_{-z}[-m]| (interior taps)
    gp = np.abs(R.template_taps([10.0], 64)[0])
    gm = np.abs(R.template_taps([-10.0], 64)[0])
    m = np.arange(-32, 32)
    inner = (m > -32) & (m < 32)
    idx = np.nonzero(inner)[0]
    assert np.max(np.abs(gp[idx] - gm[(-m[idx]) + 32])) < 1e-12


def test_retained_energy_bounded_by_parseval():
    e = R.retained_energy([0.0, 16.0, -16.0, 100.0], 256)
    assert np.all(e <= 1.0 + 1e-12)
    assert abs(e[0] - 1.0) < 1e-15          # z = 0: the delta is fully inside
    assert np.all(e[1:] > 0.99)


def test_template_spectra_is_circular_placement():
    H = R.template_spectra([4.0], 16, 64)[0]
    g = R.template_taps([4.0], 16)[0]
    # inverse DFT times L recovers the taps at m mod L
    h = np.fft.ifft(H) * 64
    m = np.arange(-8, 8)
    assert np.max(np.abs(h[m % 64] - g)) < 1e-14
    mask = np.ones(64, bool)
    mask[m % 64] = False
    assert np.max(np.abs(h[mask])) < 1e-14
