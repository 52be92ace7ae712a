"""Pins of the oracle's direct-correlation plane (oracle/direct.c).

P[j, r] = |sum_m X[r - m] g_j[m]|^2 (Section "Detailed explanation": the
spectrum is convolved with all templates to give the f-fdot plane).
"""
import math

import numpy as np
import pytest

import synth
from oracle import plane as OP
from oracle import response as R


def fft_linear_conv_power(x, g):
    """Independent brute force: full linear convolution by zero-padded FFT.
    Output index r needs conv index r + M/2 (taps start at m = -M/2)."""
    n, (nz, m) = x.size, g.shape
    L = 1 << int(math.ceil(math.log2(n + m)))
    X = np.fft.fft(x, L)
    out = np.empty((nz, n))
    for j in range(nz):
        y = np.fft.ifft(X * np.fft.fft(g[j], L))
        out[j] = np.abs(y[m // 2: m // 2 + n]) ** 2
    return out


@pytest.mark.parametrize("n,m,zs", [(300, 16, [-6.0, 0.0, 3.5]), (512, 8, [2.0]),
                                    (37, 16, [-1.0, 9.0]), (5, 4, [0.0, 1.0])])
def test_brute_force_fft_convolution(n, m, zs):
    x = synth.random_spectrum(n, seed=n + m)
    g = R.template_taps(zs, m)
    p = OP.plane(x, g)
    q = fft_linear_conv_power(x.astype(np.complex128), g)
    assert np.max(np.abs(p - q)) <= 1e-12 * max(1.0, np.max(q))


def test_zero_z_row_is_bin_power():
    x = synth.random_spectrum(4096, seed=1)
    g = R.template_taps([-4.0, 0.0, 4.0], 64)
    p = OP.plane(x, g)
    want = np.abs(x.astype(np.complex128)) ** 2
    assert np.max(np.abs(p[1] - want)) < 1e-13 * np.max(want)


def test_linearity_and_shift():
    x = synth.random_spectrum(2048, seed=2).astype(np.complex128)
    g = R.template_taps([-10.0, 7.0], 32)
    p = OP.plane(x, g)
    p2 = OP.plane(2.5 * x, g)
    assert np.allclose(p2, 6.25 * p, rtol=1e-13, atol=0)
    s = 77
    xs = np.zeros_like(x)
    xs[s:] = x[:-s]
    ps = OP.plane(xs, g)
    # away from edges (taps fully inside), P_shifted[r] = P[r - s]
    sl = slice(s + 40, x.size - 40)
    assert np.max(np.abs(ps[:, sl] - p[:, 40:x.size - 40 - s])) < 1e-12


def test_window_and_cells_agree_with_full_plane():
    x = synth.random_spectrum(1000, seed=3)
    g = R.template_taps([-2.0, 0.0, 2.0, 5.0], 16)
    full = OP.plane(x, g)
    w = OP.plane(x, g, 100, 350)
    assert np.array_equal(w, full[:, 100:350])
    j = np.array([0, 3, 2, 1])
    r = np.array([0, 999, 500, 7])
    assert np.array_equal(OP.cells(x, g, j, r), full[j, r])


def test_injected_complex_chirp_power():
    # noise-free unit complex chirp, integer mean frequency, on-grid z:
    # P(r_bar, z) = N_t * E_ret, E_ret = sum over the taps of |A(m - z/2, z)|^2
    n_t, r_bar, z, m = 1 << 14, 3000, 10.0, 64
    x = synth.complex_chirp_spectrum(n_t, r_bar - z / 2, z)
    g = R.template_taps([z], m)
    p = OP.cells(x, g, [0], [r_bar])[0]
    e_ret = R.retained_energy([z], m)[0]
    assert abs(p / (n_t * e_ret) - 1.0) < 1e-3
    # and it is the maximum of its neighbourhood in r and over a z grid
    zs = np.arange(-20.0, 41.0, 2.0)
    gg = R.template_taps(zs, m)
    blk = OP.plane(x, gg, r_bar - 20, r_bar + 21)
    jj, rr = np.unravel_index(np.argmax(blk), blk.shape)
    assert (zs[jj], rr + r_bar - 20) == (z, r_bar)


def test_real_cosine_power_quarter_amplitude_squared():
    # a real a*cos has (a/2) of the complex chirp at positive frequency
    n_t, r_bar, z, m, a = 1 << 15, 4000, -6.0, 64, 0.05
    tsamp = 1.0 / n_t
    T = 1.0
    p = synth.Pulsar(f=(r_bar - z / 2) / T, fdot=z / T ** 2, amps=[a], phases=[0.3], p1=0.0)
    x = np.zeros(n_t)
    synth.add_signal(x, tsamp, p)
    spec = synth.to_spectrum(x, sigma=1.0)
    g = R.template_taps([z], m)
    pw = OP.cells(spec, g, [0], [r_bar])[0]
    want = a * a * n_t / 4.0 * R.retained_energy([z], m)[0]
    assert abs(pw / want - 1.0) < 2e-3


def test_noise_plane_is_exp1():
    # white noise, unit-norm templates: every cell is |complex Gaussian|^2 with
    # mean 1 -> Exp(1), the chi^2_2 shape of Section "Noise properties"
    from scipy import stats
    x = synth.noise_spectrum(1 << 15, config=0, trial=7)
    zs = R.z_grid(-16, 2, 17)
    p = OP.plane(x, R.template_taps(zs, 64))
    assert abs(p.mean() - 1.0) < 0.02
    # subsample sparsely (neighbouring cells are correlated)
    s = p[::4, ::97].ravel()
    assert stats.kstest(s, "expon").pvalue > 1e-3
    assert p.max() < math.log(p.size) + 12


def test_config1_injection_peaks_at_predicted_cell():
    # f = 137.3 Hz, z = 6.4, T = 8.388608 s: r_bar = 137.3 T + 3.2 = 1154.956,
    # so the nearest cell is r = 1155 on the z = 6 row (j = 11 of -16..16 step 2)
    sp = synth.config1()
    T = sp.T
    assert abs(sp.pulsars[0].r_bar(T) - 1154.956) < 1e-3
    zs = R.z_grid(-16, 2, 17)
    g = R.template_taps(zs, 64)
    blk = OP.plane(sp.spec, g, 1135, 1176)
    jj, rr = np.unravel_index(np.argmax(blk), blk.shape)
    assert (jj, rr + 1135) == (11, 1155)
    assert blk[jj, rr] > 100.0        # matched power ~ 200 minus scalloping
