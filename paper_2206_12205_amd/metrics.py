"""Plane analysis used to grade reduced-precision planes (not on the hot path).

These are the paper's own measurements, applied to planes the library wrote:

* ``rel_diff_pct`` -- Eq. 2, the relative difference (b - s) / ((b + s) / 2)
  in percent, used for template conversion (Table 1) and peak SNRs.
* ``snr`` -- peak power divided by the standard deviation of the whole plane
  (Section "Synthetic dataset results - Power").
* ``harmonic_bands`` / ``band_maxima`` -- the plane is split into frequency
  bands from the known fundamental f (Table 3); the n-th harmonic is the
  highest cell of band n over all z (Section "Peakfinding methodology").
  Reading of the garbled caption: the fundamental band is [0, 1.5 f] closed,
  band n >= 1 is ((n + 0.5) f, (n + 1.5) f] (upper bound inclusive); ties go
  to the first cell in (z_idx, r) order.
* ``bin_match`` -- identical (r, z_idx) of band maxima between two planes
  (Section "Synthetic dataset results - Bin drift").
* ``acceleration`` -- Eq. 1, a = fdot c / f = z c / (f T^2).
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299_792_458.0


def rel_diff_pct(b, s):
    """Eq. 2: (b - s) / ((b + s) / 2) * 100, elementwise (float64)."""
    b = np.asarray(b, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    return (b - s) / (0.5 * (b + s)) * 100.0


def snr(peak_power, plane_std):
    return np.asarray(peak_power, dtype=np.float64) / float(plane_std)


def acceleration(z, f_hz, t_obs):
    """Eq. 1: acceleration in m/s^2 from drift z (bins), frequency f (Hz), T (s)."""
    return np.asarray(z, dtype=np.float64) * C_LIGHT / (f_hz * t_obs * t_obs)


def fdot_from_z(z, t_obs):
    return np.asarray(z, dtype=np.float64) / (t_obs * t_obs)


def harmonic_bands(f_hz: float, t_obs: float, n_bins: int, n_bands: int):
    """Column ranges [lo, hi) of the Table 3 bands, in Fourier bins r = f T."""
    fr = f_hz * t_obs
    out = []
    for n in range(n_bands):
        if n == 0:
            lo, hi = 0, math.floor(1.5 * fr) + 1               # [0, 1.5 f]
        else:
            lo = math.floor((n + 0.5) * fr) + 1                 # ((n+0.5) f, ...
            hi = math.floor((n + 1.5) * fr) + 1                 # ..., (n+1.5) f]
        lo, hi = max(lo, 0), min(hi, n_bins)
        if lo >= hi:
            break
        out.append((lo, hi))
    return out


def band_maxima(plane, bands):
    """For each band: (z_idx, r, power) of its highest cell over all z.

    ``plane`` is (n_z, n_bins), float32/float64 (numpy or a torch tensor on any
    device).  Ties resolve to the first cell in (z_idx, r) order."""
    res = []
    for lo, hi in bands:
        blk = plane[:, lo:hi]
        try:                                     # torch tensor
            import torch
            if isinstance(blk, torch.Tensor):
                flat = blk.contiguous().view(-1)
                mx = flat.max()
                idx = int(torch.nonzero(flat == mx)[0, 0])
                res.append((idx // (hi - lo), lo + idx % (hi - lo), float(mx)))
                continue
        except ImportError:
            pass
        b = np.asarray(blk)
        idx = int(np.argmax(b))
        res.append((idx // (hi - lo), lo + idx % (hi - lo), float(b.flat[idx])))
    return res


def bin_match(a, b):
    """Fraction of band maxima with identical (z_idx, r) in two lists."""
    if not a:
        return float("nan")
    same = sum(1 for x, y in zip(a, b) if x[0] == y[0] and x[1] == y[1])
    return same / len(a)
