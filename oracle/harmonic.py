"""Incoherent harmonic summing over the f-fdot plane (oracle).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline may use this module.

A periodic signal puts power at integer multiples of its frequency, and the
frequency derivative of harmonic h is h times the fundamental's, so harmonic
h of a signal at (r, z) sits at (h r, h z) (Section "Detailed explanation";
the paper's own analysis takes band maxima per harmonic instead of a sum,
Section "Peakfinding methodology").  The summed plane gathers the powers of
the first H harmonics onto the fundamental's cell:

  S_H[j, r] = sum_{h=1..H} P[j_h, h r],   r in [0, N_H),  N_H = floor((N - 1) / H) + 1
  z_j = z_min + j z_step,  j_h = floor((h z_j - z_min) / z_step + 1/2)

(j_h is the grid row nearest to h z_j, a tie going to the upper row).  A term
whose row j_h lies outside [0, n_z) is left out of the sum.  With a single
template (n_z = 1, no grid step) the term of harmonic h is kept (row 0) when
h z_0 equals z_0, that is z_0 = 0, and left out otherwise.

Every floating-point step of j_h is one IEEE double operation in the order
written (t = z_min + j z_step; u = h t; v = u - z_min; x = v / z_step;
j_h = floor(x + 1/2)), so any implementation that takes the same steps in
double precision lands on the same rows.  The sums are taken in double
precision over the plane values widened to double.
"""
from __future__ import annotations

import numpy as np


def n_fundamentals(n_bins: int, n_harm: int) -> int:
    """N_H: the fundamentals r whose H-th harmonic H r is a bin of the plane."""
    if n_bins < 1 or n_harm < 1:
        raise ValueError("n_bins and n_harm must be >= 1")
    return (n_bins - 1) // n_harm + 1


def harmonic_rows(z_min: float, z_step: float, n_z: int, n_harm: int) -> np.ndarray:
    """rows[j, h - 1] = j_h, or -1 where the term is left out (int64, n_z x H)."""
    rows = np.full((n_z, n_harm), -1, dtype=np.int64)
    for j in range(n_z):
        for h in range(1, n_harm + 1):
            if n_z == 1:
                zj = float(z_min)
                rows[j, h - 1] = 0 if float(h) * zj == zj else -1
                continue
            t = float(z_min) + float(j) * float(z_step)
            u = float(h) * t
            v = u - float(z_min)
            x = v / float(z_step)
            jh = int(np.floor(x + 0.5))
            rows[j, h - 1] = jh if 0 <= jh < n_z else -1
    return rows


def harmonic_sum(P: np.ndarray, z_min: float, z_step: float, n_harm: int, out_rows=None) -> np.ndarray:
    """S_H (float64, n_z x N_H) of the plane P (n_z x N); with out_rows, only
    those output rows (len(out_rows) x N_H), for sampling large planes."""
    n_z, n = P.shape
    nh = n_fundamentals(n, n_harm)
    rows = harmonic_rows(z_min, z_step, n_z, n_harm)
    r = np.arange(nh)
    want = range(n_z) if out_rows is None else list(out_rows)
    S = np.zeros((len(want), nh))
    for k, j in enumerate(want):
        for h in range(1, n_harm + 1):
            jh = rows[j, h - 1]
            if jh >= 0:
                S[k] += np.asarray(P[jh, h * r], dtype=np.float64)
    return S
