"""Pins of the jerk response and templates (oracle/response.py, w != 0).

A(q, z, w) = int_0^1 exp(i pi (2 q u + z u^2 + w u^3 / 3)) du has no closed
form; the oracle integrates it by the composite Simpson rule.  Pins: the
closed-form A(q, z) at w = 0 (a different method), the DFT of a sampled
chirp with a cubic phase (an FFT of a time series, not a quadrature),
Parseval over all integer offsets, conjugate symmetry, and the matched power
and position of an injected jerk chirp on the oracle plane.
"""
import math

import numpy as np
import pytest

import synth
from oracle import plane as OP
from oracle import response as R


@pytest.mark.parametrize("z", [0.0, 3.3, -40.0, 90.0])
def test_zero_jerk_is_the_closed_form(z):
    q = np.array([-37.2, -5.0, -0.5, 0.0, 0.25, 1.0, 7.7, 64.0])
    a = R.response_jerk(q, z, 0.0)
    b = R.response(q, z)
    assert np.max(np.abs(a - b)) < 1e-8


def test_dft_of_sampled_jerk_chirp_approaches_response():
    # the DFT of a sampled unit chirp with cubic phase, divided by N, is a
    # Riemann sum of A(r0 - k, z, w)
    n = 1 << 15
    r0, z, w = 2000.4, 20.0, -60.0
    u = np.arange(n) / n
    cyc = r0 * u + 0.5 * z * u * u + w * u ** 3 / 6.0
    x = np.exp(2j * np.pi * (cyc - np.floor(cyc)))
    X = np.fft.fft(x) / n
    k = np.arange(1985, 2035)
    a = R.response_jerk(r0 - k, z, w)
    assert np.max(np.abs(X[k] - a)) < 2e-4


@pytest.mark.parametrize("z,w,delta", [(10.0, 30.0, 0.0), (-25.0, 80.0, 0.37), (0.0, -45.0, 0.5)])
def test_parseval_over_integer_offsets(z, w, delta):
    # sum over all integer m of |A(m + delta, z, w)|^2 = int_0^1 |.|^2 = 1
    m = np.arange(-400, 401, dtype=np.float64)
    e = np.sum(np.abs(R.response_jerk(m + delta, z, w)) ** 2)
    assert abs(e - 1.0) < 2e-3


def test_conjugate_symmetry():
    q = np.array([-12.5, 0.3, 9.0])
    for z, w in ((5.0, 12.0), (-30.0, 70.0)):
        assert np.max(np.abs(R.response_jerk(q, z, w) - np.conj(R.response_jerk(-q, -z, -w)))) < 1e-9


def test_jerk_templates_unit_norm():
    g = R.template_taps([-8.0, 0.0, 6.0], 64, w=24.0)
    assert np.allclose(np.linalg.norm(g, axis=1), 1.0, atol=1e-12)


def test_injected_jerk_chirp_matched_power_and_position():
    # noise-free unit chirp with mean frequency r_bar = r0 + z/2 + w/6 on an
    # integer bin, z and w on the grid: P(r_bar, z, w) = N_t * E_ret(z, w),
    # the maximum of its neighbourhood, and well above the w = 0 plane there
    n_t, r_bar, z, w, m = 1 << 14, 3000, 10.0, 36.0, 64
    x = synth.complex_chirp_spectrum(n_t, r_bar - z / 2 - w / 6, z, w=w)
    zs = np.arange(-10.0, 31.0, 2.0)
    g = R.template_taps(zs, m, w=w)
    blk = OP.plane(x, g, r_bar - 20, r_bar + 21)
    jj, rr = np.unravel_index(np.argmax(blk), blk.shape)
    assert (zs[jj], rr + r_bar - 20) == (z, r_bar)
    e_ret = R.retained_energy([z], m, w=w)[0]
    assert abs(blk[jj, rr] / (n_t * e_ret) - 1.0) < 1e-3
    p0 = OP.plane(x, R.template_taps(zs, m), r_bar - 20, r_bar + 21)
    assert p0.max() < 0.8 * blk[jj, rr]
