"""Pins of the spectrum-preparation oracle (oracle/prep.py): the transform by
a direct DFT sum on small series, a sinusoid on an integer bin, the DC bin,
the median normaliser (noise medians land on ln 2 exactly, and the
normalised powers of white noise follow Exp(1))."""
import math

import numpy as np
import pytest

from oracle import prep


@pytest.mark.parametrize("n_t", [4, 6, 64, 250])
def test_transform_is_the_direct_dft(n_t):
    rng = np.random.default_rng(n_t)
    x = rng.normal(size=n_t)
    X = prep.prepare(x)
    t = np.arange(n_t)
    k = np.arange(n_t // 2)
    D = np.exp(-2j * np.pi * np.outer(k, t) / n_t) @ x
    D[0] = 0.0
    p = np.abs(D[1:]) ** 2
    med = np.sort(p)[(p.size - 1) // 2] if p.size % 2 else np.median(p)
    assert np.allclose(X, D / math.sqrt(med / math.log(2.0)), rtol=1e-12, atol=1e-12)


def test_sinusoid_on_an_integer_bin():
    # cos at bin 37 plus a tiny noise floor: X[37] = A n_t / 2 before scaling,
    # so the normalised |X[37]|^2 / |X[k]|^2 ratio against the noise is fixed
    n_t, k0, a = 4096, 37, 3.0
    t = np.arange(n_t)
    rng = np.random.default_rng(1)
    noise = rng.normal(size=n_t) * 1e-3
    X = prep.prepare(a * np.cos(2 * np.pi * k0 * t / n_t) + noise)
    raw = np.fft.rfft(noise)[: n_t // 2]
    med = prep.median_power(np.concatenate([[0.0], raw[1:]]))
    scale = math.sqrt(med / math.log(2.0))
    assert abs(abs(X[k0]) * scale - a * n_t / 2) < 1.0
    assert X[0] == 0.0


def test_noise_powers_are_exp1_with_median_ln2():
    rng = np.random.default_rng(5)
    X = prep.prepare(rng.normal(size=1 << 16) * 7.0)
    p = np.abs(X[1:]) ** 2
    assert abs(np.sort(p)[(p.size - 1) // 2] - math.log(2.0)) < 1e-12
    assert abs(p.mean() - 1.0) < 0.02
    assert abs(np.mean(p > 3.0) - math.exp(-3.0)) < 0.005
