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


def pulsar_windows(psr, t_obs: float, n_bins: int, z_min: float, z_step: float, n_z: int,
                   dr: int = 32, dz: float = 4.0):
    """Plane windows around one pulsar's harmonics: rows with |z - z_h| <= dz,
    columns with |r - r_h| <= dr, where r_h and z_h = h fdot T^2 are the mean
    Fourier frequency and drift of harmonic h (used where Table 3 bands of
    several pulsars overlap).  Returns (j_lo, j_hi, r_lo, r_hi), half-open."""
    out = []
    for h in range(1, len(psr.amps) + 1):
        if psr.amps[h - 1] == 0.0:
            continue
        rh, zh = psr.r_bar(t_obs, h), psr.z(t_obs, h)
        j_lo = max(int(math.ceil((zh - dz - z_min) / z_step)), 0)
        j_hi = min(int(math.floor((zh + dz - z_min) / z_step)) + 1, n_z)
        r_lo = max(int(math.floor(rh - dr)), 0)
        r_hi = min(int(math.floor(rh + dr)) + 1, n_bins)
        if j_lo < j_hi and r_lo < r_hi:
            out.append((j_lo, j_hi, r_lo, r_hi))
    return out


def window_maxima(plane, windows):
    """For each window (j_lo, j_hi, r_lo, r_hi): (z_idx, r, power) of its
    highest cell; ties resolve to the first cell in (z_idx, r) order."""
    res = []
    for j_lo, j_hi, r_lo, r_hi in windows:
        blk = plane[j_lo:j_hi, r_lo:r_hi]
        w = r_hi - r_lo
        try:
            import torch
            if isinstance(blk, torch.Tensor):
                flat = blk.contiguous().view(-1)
                mx = flat.max()
                idx = int(torch.nonzero(flat == mx)[0, 0])
                res.append((j_lo + idx // w, r_lo + idx % w, float(mx)))
                continue
        except ImportError:
            pass
        b = np.asarray(blk)
        idx = int(np.argmax(b))
        res.append((j_lo + idx // w, r_lo + idx % w, float(b.flat[idx])))
    return res
