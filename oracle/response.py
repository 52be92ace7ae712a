"""Acceleration response and template bank, double precision (oracle).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline may use this module.

The paper builds its correlation templates from the Fourier response of a
linearly drifting sinusoid, citing Ransom et al. 2002 for the method (Section
"Introduction"; Section "Template conversion" shows the template magnitudes
only as a figure).  The formula is therefore derived here from first
principles rather than taken from the text.

Response.  A unit complex chirp exp(2 pi i (r0 u + z u^2 / 2)), u = t / T in
[0, 1), has normalised DFT value at bin k

    A(q, z) = integral_0^1 exp(i pi (2 q u + z u^2)) du,    q = r0 - k,

where z is the drift in Fourier bins over the observation (Eq. 1).  For z > 0,
completing the square gives, with Y1 = q sqrt(2/z), Y2 = (q + z) sqrt(2/z) and
E(x) = C(x) + i S(x) the Fresnel integrals,

    A = exp(-i pi q^2 / z) / sqrt(2 z) * (E(Y2) - E(Y1)).

When Y1 and Y2 have the same sign the large phases cancel analytically: with
G(x) = (1 + i)/2 * erfcx(sqrt(pi)/2 (1 - i) x) (x >= 0), E(x) = (1+i)/2 -
G(x) exp(i pi x^2 / 2), so

    Y1 >= 0:  A = (G(Y1) - G(Y2) exp(i pi (2q + z))) / sqrt(2 z)
    Y2 <= 0:  A = (G(-Y2) exp(i pi (2q + z)) - G(-Y1)) / sqrt(2 z).

z < 0 follows from A(q, z) = conj(A(-q, -z)); z = 0 is Fourier interpolation,
A(q, 0) = exp(i pi q) sin(pi q) / (pi q).  For 0 < |z| < 1e-3 the oracle
integrates the definition directly by composite Gauss-Legendre quadrature.

Templates.  Reading of the paper's silent points (r is the *mean* Fourier
frequency; M taps m in [-M/2, M/2); unit l2 norm after truncation):

    g_z[m] = conj(A(m - z/2, z)) / ||.||_2,

and the plane is P[z, r] = |sum_m X[r - m] g_z[m]|^2 (X = 0 outside [0, N)).
The overlap-save form needs the length-L spectrum of the circularly placed
taps, H_z = FFT_L(h_z) / L with h_z[m mod L] = g_z[m]; the 1/L folds the
inverse transform's normalisation into the template.

Jerk.  A third search axis (Section "FDAS vs Jerk Search" describes it; the
paper studies z only): a
sinusoid whose drift changes by w bins over the observation has response
A(q, z, w) = integral_0^1 exp(i pi (2 q u + z u^2 + w u^3 / 3)) du, taken
here by the composite Simpson rule (response_jerk), and templates
g[m] = conj(A(m - z/2 - w/6, z, w)) / ||.||.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfcx, fresnel

_SMALL_Z = 1e-3


def _gl_nodes(n: int = 16):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w          # on [0, 1]


def quad_moment(q, z, power: int = 0):
    """integral_0^1 u^power exp(i pi (2 q u + z u^2)) du by composite
    16-point Gauss-Legendre; panels resolve every half oscillation."""
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    q, z = np.broadcast_arrays(q, z)
    out = np.empty(q.shape, dtype=np.complex128)
    xg, wg = _gl_nodes(16)
    flat_q, flat_z, flat_o = q.ravel(), z.ravel(), out.reshape(-1)
    npan = np.ceil(2.0 * (np.abs(flat_q) + np.abs(flat_z))).astype(np.int64) + 2
    for n in np.unique(npan):
        sel = np.nonzero(npan == n)[0]
        edges = np.arange(n, dtype=np.float64) / n
        u = (edges[:, None] + xg[None, :] / n).ravel()          # nodes
        w = np.tile(wg / n, n)
        # process in blocks to bound memory
        for s in range(0, sel.size, 4096):
            idx = sel[s:s + 4096]
            ph = np.pi * (2.0 * flat_q[idx, None] * u[None, :]
                          + flat_z[idx, None] * u[None, :] ** 2)
            f = np.exp(1j * ph) * (w * u ** power)[None, :]
            flat_o[idx] = f.sum(axis=1)
    return out


def _E(x):
    s, c = fresnel(x)          # scipy returns (S, C)
    return c + 1j * s


def _G(x):
    """(1 + i)/2 * erfcx(sqrt(pi)/2 (1 - i) x), x >= 0."""
    return (0.5 + 0.5j) * erfcx((0.5 * math.sqrt(math.pi)) * (1.0 - 1.0j) * x)


def _response_pos(q, z):
    """Closed form for z > 0 (arrays of equal shape)."""
    s = np.sqrt(2.0 / z)
    y1 = q * s
    y2 = (q + z) * s
    rt = np.sqrt(2.0 * z)
    out = np.empty(q.shape, dtype=np.complex128)
    # exp(i pi (2q + z)) with the argument reduced mod 2 exactly enough
    ph = np.mod(2.0 * q + z, 2.0)
    e = np.exp(1j * np.pi * ph)
    pos = y1 >= 0.0
    neg = y2 <= 0.0
    mid = ~(pos | neg)
    if pos.any():
        out[pos] = (_G(y1[pos]) - _G(y2[pos]) * e[pos]) / rt[pos]
    if neg.any():
        out[neg] = (_G(-y2[neg]) * e[neg] - _G(-y1[neg])) / rt[neg]
    if mid.any():
        qm, zm = q[mid], z[mid]
        out[mid] = (np.exp(-1j * np.pi * np.mod(qm * qm / zm, 2.0))
                    / rt[mid] * (_E(y2[mid]) - _E(y1[mid])))
    return out


def response(q, z):
    """A(q, z) = integral_0^1 exp(i pi (2 q u + z u^2)) du, complex128."""
    q = np.asarray(q, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    q, z = np.broadcast_arrays(q, z)
    out = np.empty(q.shape, dtype=np.complex128)
    zero = z == 0.0
    small = (~zero) & (np.abs(z) < _SMALL_Z)
    pos = z >= _SMALL_Z
    neg = z <= -_SMALL_Z
    if zero.any():
        qq = q[zero]
        out[zero] = np.exp(1j * np.pi * np.mod(qq, 2.0)) * np.sinc(qq)
    if small.any():
        out[small] = quad_moment(q[small], z[small], 0)
    if pos.any():
        out[pos] = _response_pos(q[pos], z[pos])
    if neg.any():
        out[neg] = np.conj(_response_pos(-q[neg], -z[neg]))
    return out


def response_grad(q, z):
    """(dA/dq, dA/dz) at fixed q, by quadrature of the differentiated integrand:
    dA/dq = int 2 pi i u e^{...} du,  dA/dz = int i pi u^2 e^{...} du."""
    dq = 2j * np.pi * quad_moment(q, z, 1)
    dz = 1j * np.pi * quad_moment(q, z, 2)
    return dq, dz


def response_jerk(q, z, w, phase_step: float = 0.02) -> np.ndarray:
    """A(q, z, w) = integral_0^1 exp(i pi (2 q u + z u^2 + w u^3 / 3)) du.

    A sinusoid whose frequency runs r0 + z u + w u^2 / 2 over the observation
    (w: the change of the drift, the jerk search's third axis).  No closed
    form: composite Simpson rule on an even number of intervals, each at most
    phase_step radians of phase (|phase'| <= pi (2|q| + 2|z| + |w|)), so the
    rule's error (h phase')^4 / 180 stays near 1e-9."""
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    w = np.atleast_1d(np.asarray(w, dtype=np.float64))
    q, z, w = np.broadcast_arrays(q, z, w)
    out = np.empty(q.shape, dtype=np.complex128)
    for idx in np.ndindex(q.shape):
        qq, zz, ww = q[idx], z[idx], w[idx]
        rate = math.pi * (2.0 * abs(qq) + 2.0 * abs(zz) + abs(ww))
        n = max(64, 2 * int(math.ceil(rate / phase_step / 2.0)))
        u = np.linspace(0.0, 1.0, n + 1)
        f = np.exp(1j * math.pi * (2.0 * qq * u + zz * u * u + ww * u ** 3 / 3.0))
        coef = np.ones(n + 1)
        coef[1:-1:2] = 4.0
        coef[2:-1:2] = 2.0
        out[idx] = np.dot(coef, f) / (3.0 * n)
    return out


def z_grid(z_min: float, z_step: float, n_z: int) -> np.ndarray:
    return z_min + z_step * np.arange(n_z, dtype=np.float64)


def template_taps(zs, n_taps: int, normalise: bool = True, w: float = 0.0) -> np.ndarray:
    """g_z[m] for m in [-M/2, M/2), rows per z, column i = m + M/2 (complex128).
    With a jerk w: g_z[m] = conj(A(m - z/2 - w/6, z, w)) / ||.|| (r stays the
    mean frequency r0 + z/2 + w/6)."""
    if n_taps % 2:
        raise ValueError("n_taps must be even")
    zs = np.atleast_1d(np.asarray(zs, dtype=np.float64))
    m = np.arange(-n_taps // 2, n_taps // 2, dtype=np.float64)
    if w == 0.0:
        g = np.conj(response(m[None, :] - 0.5 * zs[:, None], zs[:, None]))
    else:
        g = np.conj(response_jerk(m[None, :] - 0.5 * zs[:, None] - w / 6.0, zs[:, None], w))
    if normalise:
        g /= np.linalg.norm(g, axis=1, keepdims=True)
    return g


def retained_energy(zs, n_taps: int, w: float = 0.0) -> np.ndarray:
    """sum over the M taps of |A(m - z/2 - w/6, z, w)|^2 (Parseval: 1 over all m)."""
    g = template_taps(zs, n_taps, normalise=False, w=w)
    return np.sum(np.abs(g) ** 2, axis=1)


def template_spectra(zs, n_taps: int, seg_len: int, w: float = 0.0) -> np.ndarray:
    """H_z = FFT_L(h_z) / L with h_z[m mod L] = g_z[m]; rows per z, complex128."""
    if seg_len <= n_taps:
        raise ValueError("segment length must exceed the tap count")
    g = template_taps(zs, n_taps, w=w)
    h = np.zeros((g.shape[0], seg_len), dtype=np.complex128)
    m = np.arange(-n_taps // 2, n_taps // 2)
    h[:, np.mod(m, seg_len)] = g
    return np.fft.fft(h, axis=1) / seg_len
