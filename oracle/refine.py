"""Interpolated correlation power at continuous (r, z) and its gradient (oracle).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline may use this module.

The plane samples the matched-filter power on an integer r grid and a discrete
z grid; quantisation in both axes moves peaks into adjacent bins (Section
"Peakfinding methodology").  Candidate refinement evaluates the same matched
filter at continuous (r, z) from a window of K spectral bins around r:

    F(r, z) = sum_{k = floor(r) - K/2 + 1}^{floor(r) + K/2} X[k] conj(A(r - z/2 - k, z)),
    P(r, z) = |F|^2 ,

with A the acceleration response (mean-frequency convention, as the
templates) and X = 0 outside [0, N).  Its gradient is

    dP/dr = 2 Re(conj(F) dF/dr),  dF/dr = sum X[k] conj(A_q),
    dP/dz = 2 Re(conj(F) dF/dz),  dF/dz = sum X[k] conj(A_z - A_q / 2),

where A_q, A_z are the partial derivatives at fixed q, computed here by
Gauss-Legendre quadrature of the differentiated integrand (independent of the
closed-form derivatives a GPU kernel would use).

Ascent step (reading; the paper prints no refinement): a Newton step on the
analytic curvature of an isolated peak, d2P/dr2 = -2 pi^2 P / 3 and
d2P/dz2 = -pi^2 P / 90, i.e. r += eta_r dP/dr, z += eta_z dP/dz with
eta_r = s_r * 3 / (2 pi^2 P) and eta_z = s_z * 90 / (pi^2 P).
"""
from __future__ import annotations

import math

import numpy as np

from .response import response, response_grad


def _window(spec, r, taps):
    x = np.asarray(spec, dtype=np.complex128)
    n = x.size
    base = np.floor(r).astype(np.int64)
    k = base[:, None] + np.arange(-taps // 2 + 1, taps // 2 + 1)[None, :]
    inside = (k >= 0) & (k < n)
    xv = np.where(inside, x[np.clip(k, 0, n - 1)], 0.0)
    return k, xv


def power(spec, r, z, taps: int = 32):
    """P(r, z) and the complex amplitude F (float64 / complex128 arrays)."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    k, xv = _window(spec, r, taps)
    q = r[:, None] - 0.5 * z[:, None] - k
    F = np.sum(xv * np.conj(response(q, np.broadcast_to(z[:, None], q.shape))), axis=1)
    return np.abs(F) ** 2, F


def power_grad(spec, r, z, taps: int = 32):
    """(P, dP/dr, dP/dz) at continuous (r, z), float64."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    k, xv = _window(spec, r, taps)
    q = r[:, None] - 0.5 * z[:, None] - k
    zz = np.broadcast_to(z[:, None], q.shape)
    A = response(q, zz)
    Aq, Az = response_grad(q, zz)
    F = np.sum(xv * np.conj(A), axis=1)
    Fr = np.sum(xv * np.conj(Aq), axis=1)
    Fz = np.sum(xv * np.conj(Az - 0.5 * Aq), axis=1)
    P = np.abs(F) ** 2
    dPr = 2.0 * np.real(np.conj(F) * Fr)
    dPz = 2.0 * np.real(np.conj(F) * Fz)
    return P, dPr, dPz


def ascend(spec, r, z, steps: int = 20, taps: int = 32,
           eta_r_scale: float = 1.0, eta_z_scale: float = 1.0):
    """Gradient ascent; returns final (r, z, P, dP/dr, dP/dz)."""
    r = np.array(r, dtype=np.float64)
    z = np.array(z, dtype=np.float64)
    for _ in range(steps):
        P, gr, gz = power_grad(spec, r, z, taps)
        Ps = np.maximum(P, 1e-30)
        r = r + eta_r_scale * 3.0 / (2.0 * math.pi ** 2 * Ps) * gr
        z = z + eta_z_scale * 90.0 / (math.pi ** 2 * Ps) * gz
    P, gr, gz = power_grad(spec, r, z, taps)
    return r, z, P, gr, gz
