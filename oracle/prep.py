"""Spectrum preparation upstream of the correlation (oracle).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline may use this module.

The correlation takes a normalised complex spectrum.  The paper keeps the
real FFT that makes it in single precision (Section "Casting between
single-precision and bfloat16" and the pipeline description) and normalises
the spectrum by its median power.  The reading used here:

  X[k] = sum_t x[t] exp(-2 pi i k t / N_t),    k in [0, N_t / 2)
         (the Nyquist bin k = N_t / 2 is dropped)
  X[0] = 0                                       (the DC bin carries no signal)
  X[k] /= sqrt(median_{k >= 1} |X[k]|^2 / ln 2)

so that white-noise powers |X[k]|^2 become Exp(1) (their median is ln 2).
The transform is the library FFT in double precision, the median the middle
element of the sorted powers (N_t / 2 - 1 of them: an odd count when N_t is
a multiple of 4; otherwise the mean of the two middle elements).
"""
from __future__ import annotations

import math

import numpy as np


def prepare(x: np.ndarray) -> np.ndarray:
    """Normalised spectrum (complex128, N_t / 2 bins) of the real series x."""
    x = np.asarray(x, dtype=np.float64)
    n_t = x.size
    if n_t < 4 or n_t % 2:
        raise ValueError("the series needs an even length >= 4")
    X = np.fft.rfft(x)[: n_t // 2]
    X[0] = 0.0
    p = np.sort(X[1:].real ** 2 + X[1:].imag ** 2)
    med = p[(p.size - 1) // 2] if p.size % 2 else 0.5 * (p[p.size // 2 - 1] + p[p.size // 2])
    return X / math.sqrt(med / math.log(2.0))


def median_power(X: np.ndarray) -> float:
    """The median of |X[k]|^2 over k >= 1 (the normaliser's argument)."""
    p = np.sort(np.abs(np.asarray(X[1:])) ** 2)
    return float(p[(p.size - 1) // 2] if p.size % 2 else 0.5 * (p[p.size // 2 - 1] + p[p.size // 2]))
