"""Pins of the oracle's peak finder and bfloat16 cast."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import casts, peaks
from oracle import response as R
from paper_2206_12205_amd import metrics

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def brute_peaks(P, thr):
    """Pure-Python loops over every cell and neighbour (tiny planes only)."""
    nz, n = P.shape
    out = []
    for j in range(nz):
        for r in range(n):
            c = P[j, r]
            if not c > thr:
                continue
            ok = True
            for dj in (-1, 0, 1):
                for dr in (-1, 0, 1):
                    if dj == 0 and dr == 0:
                        continue
                    a, b = j + dj, r + dr
                    if not (0 <= a < nz and 0 <= b < n):
                        continue
                    before = (a, b) < (j, r)
                    if before and not c > P[a, b]:
                        ok = False
                    if not before and not c >= P[a, b]:
                        ok = False
            if ok:
                out.append((j, r))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_peaks_brute_force_with_ties(seed):
    g = np.random.default_rng(seed)
    P = g.integers(0, 5, size=(7, 40)).astype(np.float32)   # many ties
    j, r, p = peaks.peaks(P, 1.5, rows_per_block=3)
    assert list(zip(j.tolist(), r.tolist())) == brute_peaks(P, 1.5)
    assert np.array_equal(p, P[j, r])


def test_peaks_fixtures():
    P = np.zeros((3, 6))
    P[1, 2] = P[1, 3] = 9.0          # plateau: the first cell in row-major order wins
    P[0, 0] = 5.0                    # corner peak
    P[2, 5] = 4.0                    # below threshold 4.5 -> not a peak
    P[2, 0] = np.nan                 # NaN is never a peak
    j, r, _ = peaks.peaks(P, 4.5)
    assert list(zip(j.tolist(), r.tolist())) == [(0, 0), (1, 2)]
    # vertical plateau: upper cell precedes the lower one
    Q = np.zeros((4, 4))
    Q[1, 1] = Q[2, 1] = 3.0
    j, r, _ = peaks.peaks(Q, 1.0)
    assert list(zip(j.tolist(), r.tolist())) == [(1, 1)]


def test_bf16_rne_exact_cases():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)            # bf16 spacing at 1.0
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20,
                     -2.5, 3.0e38, 1e-40, 0.0], dtype=np.float32)
    b = casts.to_bf16(vals)
    assert b[0] == one
    assert b[1] == one                     # tie -> even (1.0)
    assert b[2] == one + 2 * ulp           # tie -> even (1 + 2^-6)
    assert b[3] == one + ulp               # above the tie -> up
    assert b[4] == np.float32(-2.5)
    assert np.isfinite(b[5])
    assert np.isnan(casts.to_bf16(np.array([np.nan], np.float32)))[0]
    # widening is exact: bits << 16
    bits = casts.bf16_bits(vals)
    assert np.array_equal(casts.bf16_widen(bits).view(np.uint32) & 0xFFFF, np.zeros(8, np.uint32))


def test_bf16_template_conversion_matches_table1():
    """Eq. 2 statistics of fp32 -> bf16 template conversion (Table 1): RNE
    reproduces |rel diff| <= ~0.39 %, mean ~ 0, sigma ~ 0.15 %; truncation
    does not (it is biased to about -0.2 % and reaches -0.78 %)."""
    with open(os.path.join(GOLD, "table1_template_conversion.json")) as f:
        t1 = json.load(f)
    H = R.template_spectra(R.z_grid(-100, 2, 101), 256, 8192)
    for part, key in ((H.real, "real"), (H.imag, "imaginary")):
        s = part.astype(np.float32).ravel()
        s = s[np.abs(s) > 1e-30]
        d = metrics.rel_diff_pct(casts.to_bf16(s), s)
        ref = t1[key]
        assert d.max() <= ref["max_pct"] + 0.003
        assert d.min() >= ref["min_pct"] - 0.003
        assert abs(d.mean()) < 0.01
        assert 0.10 < d.std() < 0.20            # Table 1: ~0.153 %
        dt = metrics.rel_diff_pct(casts.bf16_truncate(s), s)
        assert dt.mean() < -0.1 or dt.min() < ref["min_pct"] - 0.1


def test_eq2_and_units():
    assert metrics.rel_diff_pct(101.0, 99.0) == pytest.approx(2.0)
    assert metrics.rel_diff_pct(1.0, 1.0) == 0.0
    # Eq. 1: a = z c / (f T^2); z = 0.5, f = 463.097 Hz, T = 345 s
    a = float(metrics.acceleration(0.5, 463.097, 345.0))
    assert a == pytest.approx(0.5 * 299792458.0 / (463.097 * 345.0 ** 2))
    assert metrics.fdot_from_z(2.0, 2.0) == pytest.approx(0.5)


def test_bands_table3():
    # f T = 100 bins: fundamental [0, 150], band 1 (150, 250], band 2 (250, 350]
    b = metrics.harmonic_bands(10.0, 10.0, 10_000, 3)
    assert b == [(0, 151), (151, 251), (251, 351)]
    P = np.zeros((3, 400))
    P[2, 150] = 5.0
    P[0, 151] = 7.0
    P[1, 300] = 7.0
    P[0, 300] = 7.0                  # tie with (1, 300): first in (z, r) order wins
    mx = metrics.band_maxima(P, b)
    assert mx == [(2, 150, 5.0), (0, 151, 7.0), (0, 300, 7.0)]
    assert metrics.bin_match(mx, mx) == 1.0


def test_e4m3_table_and_rounding():
    """OCP e4m3fn: spot values of the format definition, round-trip of every
    finite code, ties to even, subnormals, NaN."""
    from oracle import casts as C
    v = C.E4M3_TABLE
    assert v[0x7E] == 448.0 and v[0x38] == 1.0 and v[0x40] == 2.0
    assert v[0x08] == 2.0 ** -6 and v[0x01] == 2.0 ** -9 and v[0x00] == 0.0
    assert np.isnan(v[0x7F]) and np.isnan(v[0xFF]) and v[0xB8] == -1.0
    finite = [c for c in range(256) if not np.isnan(v[c]) and c != 0x80]
    assert np.array_equal(C.e4m3_bits(v[finite]), np.array(finite, dtype=np.uint8))
    # monotone over the non-negative codes
    assert np.all(np.diff(v[:0x7F]) > 0)
    # ties to even: 1 + 1/16 lies between codes 0x38 (1.0) and 0x39 (1.125)
    assert C.e4m3_bits(1.0625) == 0x38 and C.e4m3_bits(1.1875) == 0x3A
    assert C.e4m3_bits(1.0626) == 0x39 and C.e4m3_bits(-1.0625) == 0xB8
    # subnormal ties: 1.5 * 2^-9 lies between 0x01 and 0x02 -> 0x02 (even)
    assert C.e4m3_bits(1.5 * 2.0 ** -9) == 0x02 and C.e4m3_bits(0.5 * 2.0 ** -9) == 0x00
    assert C.e4m3_bits(460.0) == 0x7E and C.e4m3_bits(464.0) == 0x7F
    assert C.e4m3_bits(float("nan")) == 0x7F
    # nearest: relative error at most 2^-4 over the normal range
    g = np.random.default_rng(3)
    x = np.exp(g.uniform(np.log(2.0 ** -6), np.log(448.0), 2000))
    r = C.to_e4m3(x)
    assert np.max(np.abs(r - x) / x) <= 2.0 ** -4 + 1e-15


def test_band_max_against_brute_force_with_ties_nan_and_clipping():
    """Band maxima vs a pure-Python scan in (z, r) order (ties: first cell;
    NaN skipped; windows clipped at the plane's edges; empty windows)."""
    from oracle import peaks as OPK
    rng = np.random.default_rng(7)
    P = np.round(rng.uniform(0, 4, size=(9, 57)))          # few distinct values: many ties
    P[3, 10:20] = np.nan
    P[0:2, 50:57] = np.nan
    windows = [(0, 9, 0, 57), (2, 5, 8, 22), (-3, 2, 48, 70), (0, 2, 50, 57), (4, 4, 0, 10),
               (7, 20, -5, 3), (3, 4, 10, 20), (1, 8, 30, 31)]
    z, r, p = OPK.band_max(P, windows)
    for k, (z_lo, z_hi, r_lo, r_hi) in enumerate(windows):
        best = None
        for zz in range(max(z_lo, 0), min(z_hi, 9)):
            for cc in range(max(r_lo, 0), min(r_hi, 57)):
                v = P[zz, cc]
                if v != v:
                    continue
                if best is None or v > best[2]:
                    best = (zz, cc, v)
        if best is None:
            assert (z[k], r[k]) == (-1, -1) and np.isnan(p[k])
        else:
            assert (z[k], r[k], p[k]) == best


# --- margins: pinned by hand-built planes and by what a margin means --------

def test_margins_hand_built():
    """Gaps worked out by hand: threshold gap, gap to each of the 8
    neighbours, edge and corner cells, and the max(P, 1) floor."""
    P = np.array([[1.0, 2.0, 3.0, 0.0],
                  [4.0, 10.0, 7.5, 0.0],
                  [0.0, 9.0, 2.0, 0.25]])
    # centre cell 10 (thr 6): threshold gap 4; nearest neighbour 9 (below
    # it, a following neighbour) -> gap 1 -> 1 / 10
    # corner (0, 0) = 1 (thr 0.5): neighbours 2, 4, 10 -> gaps 1, 3, 9;
    # threshold gap 0.5 is the smallest; floor max(1, 1) = 1
    # edge (0, 2) = 3 (thr 0): neighbours 2, 0, 10, 7.5, 0 -> smallest |3 - 2| = 1
    # corner (2, 3) = 0.25 (thr 0.2): threshold gap 0.05, neighbours 7.5, 0,
    # 2 -> 0.25; floor max(0.25, 1) = 1 -> 0.05 (not 0.05 / 0.25)
    got = peaks.margins(P, [1, 0, 0, 2], [1, 0, 2, 3], 6.0)
    assert got[0] == pytest.approx(0.1, abs=1e-15)
    assert peaks.margins(P, [0], [0], 0.5)[0] == pytest.approx(0.5, abs=1e-15)
    assert peaks.margins(P, [0], [2], 0.0)[0] == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert peaks.margins(P, [2], [3], 0.2)[0] == pytest.approx(0.05, abs=1e-15)
    # each of the 8 neighbours in turn is the closest one
    for dj in (-1, 0, 1):
        for dr in (-1, 0, 1):
            if dj == 0 and dr == 0:
                continue
            Q = np.full((3, 3), 1.0)
            Q[1, 1] = 8.0
            Q[1 + dj, 1 + dr] = 7.75
            assert peaks.margins(Q, [1], [1], 2.0)[0] == pytest.approx(0.25 / 8.0, abs=1e-15), (dj, dr)
    # threshold gap smaller than every neighbour gap
    Q = np.full((3, 3), 1.0)
    Q[1, 1] = 8.0
    assert peaks.margins(Q, [1], [1], 7.9)[0] == pytest.approx(0.1 / 8.0, abs=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_margins_is_the_decrease_that_removes_a_peak(seed):
    """For every peak the margin m is the smallest relative decrease that
    un-peaks it: lowering the cell by 0.999 m max(P, 1) keeps it a peak,
    lowering it by 1.001 m max(P, 1) removes it (it falls to the threshold or
    to a neighbour).  Checked through the peak finder, edges and corners
    included."""
    g = np.random.default_rng(100 + seed)
    P = np.round(g.exponential(2.0, size=(5, 9)), 2) + g.uniform(0, 1e-3, size=(5, 9))
    if seed % 2:
        P *= 0.3                      # many cells below 1: the max(P, 1) floor matters
    thr = float(np.quantile(P, 0.4))
    j, r, _ = peaks.peaks(P, thr)
    assert len(j) > 0
    m = peaks.margins(P, j, r, thr)
    assert np.all(m > 0)
    for jj, rr, mm in zip(j, r, m):
        step = mm * max(P[jj, rr], 1.0)
        for f, stays in ((0.999, True), (1.001, False)):
            Q = P.copy()
            Q[jj, rr] -= f * step
            qj, qr, _ = peaks.peaks(Q, thr)
            assert ((jj, rr) in set(zip(qj.tolist(), qr.tolist()))) == stays, (jj, rr, f)
