"""Thresholded peak finding on the f-fdot plane (oracle).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline may use this module.

A pulsar appears on the plane as a peak (Section "Detailed explanation").  The
paper does not describe its peak finder, so the reading used here is:

  cell (j, r) is a peak  iff  P[j, r] > threshold,
                              P[j, r] >  each existing neighbour that precedes
                                          it in row-major (j, r) order,
                              P[j, r] >= each existing neighbour that follows it,

over the 8-neighbourhood (edge cells compare only the neighbours that exist).
Exactly one cell of a plateau of equal maxima is reported (its first cell).
Peaks are listed sorted by (j, r).  NaN never compares true, so NaN cells are
never peaks.
"""
from __future__ import annotations

import numpy as np

_PRECEDING = [(-1, -1), (-1, 0), (-1, 1), (0, -1)]
_FOLLOWING = [(0, 1), (1, -1), (1, 0), (1, 1)]


def _block_peaks(P, thr, j_lo, j_hi):
    """Peaks with rows in [j_lo, j_hi) of the full plane P."""
    n_z, n = P.shape
    a, b = max(j_lo - 1, 0), min(j_hi + 1, n_z)
    blk = np.asarray(P[a:b], dtype=np.float64)
    pad = np.full((blk.shape[0] + 2, n + 2), -np.inf)
    pad[1:-1, 1:-1] = blk
    c0 = j_lo - a                      # first owned row inside blk
    rows = j_hi - j_lo
    c = blk[c0:c0 + rows]
    ok = c > thr
    for dj, dr in _PRECEDING:
        nb = pad[1 + c0 + dj:1 + c0 + dj + rows, 1 + dr:1 + dr + n]
        ok &= c > nb
    for dj, dr in _FOLLOWING:
        nb = pad[1 + c0 + dj:1 + c0 + dj + rows, 1 + dr:1 + dr + n]
        ok &= c >= nb
    jj, rr = np.nonzero(ok)
    return jj + j_lo, rr, c[jj, rr]


def peaks(P, threshold: float, rows_per_block: int = 8):
    """Return (z_idx int32, r int64, power float64), sorted by (z_idx, r)."""
    n_z = P.shape[0]
    js, rs, ps = [], [], []
    for j0 in range(0, n_z, rows_per_block):
        j, r, p = _block_peaks(P, threshold, j0, min(j0 + rows_per_block, n_z))
        js.append(j)
        rs.append(r)
        ps.append(p)
    if not js:
        return (np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(0))
    return (np.concatenate(js).astype(np.int32), np.concatenate(rs).astype(np.int64),
            np.concatenate(ps))


def margins(P, j, r, threshold: float):
    """Smallest relative gap of each listed cell to the threshold and to its
    neighbours: min(|P - thr|, |P - nb|) / max(P, 1).  Peaks whose margin is
    below the comparison tolerance are ambiguous between precisions."""
    n_z, n = P.shape
    out = np.empty(len(j))
    for i, (jj, rr) in enumerate(zip(j, r)):
        c = float(P[jj, rr])
        gap = abs(c - threshold)
        for dj in (-1, 0, 1):
            for dr in (-1, 0, 1):
                if dj == 0 and dr == 0:
                    continue
                a, b = jj + dj, rr + dr
                if 0 <= a < n_z and 0 <= b < n:
                    gap = min(gap, abs(c - float(P[a, b])))
        out[i] = gap / max(c, 1.0)
    return out


def band_max(P, windows):
    """Highest cell of each window (z_lo, z_hi, r_lo, r_hi), half-open and
    clipped to the plane: the paper's peak-finding method takes the highest
    point of each harmonic band (Section "Peakfinding methodology", Table 3).
    NaN cells are skipped; ties go to the first cell in (z_idx, r) order.
    Returns (z_idx int64, r int64, power float64); a window with no
    non-NaN cell gives (-1, -1, nan)."""
    n_z, n = P.shape
    zs, rs, ps = [], [], []
    for z_lo, z_hi, r_lo, r_hi in windows:
        a, b = max(int(z_lo), 0), min(int(z_hi), n_z)
        c, d = max(int(r_lo), 0), min(int(r_hi), n)
        best = None
        if a < b and c < d:
            blk = np.asarray(P[a:b, c:d], dtype=np.float64)
            ok = ~np.isnan(blk)
            if ok.any():
                m = np.max(blk[ok])
                jj, rr = np.nonzero(ok & (blk == m))      # row-major order: the first is the tie winner
                best = (a + int(jj[0]), c + int(rr[0]), float(m))
        if best is None:
            best = (-1, -1, float("nan"))
        zs.append(best[0])
        rs.append(best[1])
        ps.append(best[2])
    return np.array(zs, np.int64), np.array(rs, np.int64), np.array(ps)
