"""Pins of the harmonic-summing oracle (oracle/harmonic.py).

S_H[j, r] = sum_h P[j_h, h r] with j_h the grid row nearest to h z_j.  Each
pin fixes the result by a route other than the oracle's own loops: counts of
in-range harmonics by inequalities, the cells a single bright cell reaches
by divisor enumeration, the tie rule on a grid where h z_j falls halfway, and
the physics of a harmonic series of chirps whose matched powers are known in
closed form.
"""
import numpy as np
import pytest

import synth
from oracle import harmonic as HS
from oracle import plane as OP
from oracle import response as R


def test_one_harmonic_is_the_plane():
    rng = np.random.default_rng(1)
    P = rng.exponential(size=(7, 101))
    S = HS.harmonic_sum(P, -6.0, 2.0, 1)
    assert S.shape == P.shape and np.array_equal(S, P)


@pytest.mark.parametrize("n_harm", [2, 3, 4, 8, 16])
def test_all_ones_plane_counts_in_range_harmonics(n_harm):
    # symmetric integer grid z_j = 2 (j - 50): harmonic h of row j sits on
    # row 50 + h (j - 50), inside [0, 101) iff h |j - 50| <= 50
    n_z, n = 101, 1000
    S = HS.harmonic_sum(np.ones((n_z, n)), -100.0, 2.0, n_harm)
    assert S.shape == (n_z, (n - 1) // n_harm + 1)
    for j in range(n_z):
        d = abs(j - 50)
        want = n_harm if d == 0 else min(n_harm, 50 // d)
        assert np.all(S[j] == want), j


@pytest.mark.parametrize("i0,c0", [(50, 360), (62, 360), (40, 97), (0, 840), (100, 7)])
def test_single_cell_reaches_its_divisor_cells(i0, c0):
    n_z, n, H = 101, 1000, 8
    P = np.zeros((n_z, n))
    P[i0, c0] = 1.0
    S = HS.harmonic_sum(P, -100.0, 2.0, H)
    want = np.zeros_like(S)
    for h in range(1, H + 1):
        if c0 % h or (i0 - 50) % h:
            continue
        r, j = c0 // h, 50 + (i0 - 50) // h
        if r < S.shape[1]:
            want[j, r] += 1.0
    assert np.array_equal(S, want)


def test_tie_goes_to_the_upper_row():
    # z_j = -3 + 2 j: 2 z_j = -6 + 4 j lies halfway between rows 2 j - 2 and
    # 2 j - 1, and 3 z_j = -9 + 6 j lies on row 3 j - 3
    rows = HS.harmonic_rows(-3.0, 2.0, 12, 3)
    for j in range(12):
        assert rows[j, 0] == j
        assert rows[j, 1] == (2 * j - 1 if 0 <= 2 * j - 1 < 12 else -1)
        assert rows[j, 2] == (3 * j - 3 if 0 <= 3 * j - 3 < 12 else -1)


def test_single_template_keeps_only_its_own_row():
    rng = np.random.default_rng(2)
    P = rng.exponential(size=(1, 64))
    S0 = HS.harmonic_sum(P, 0.0, 0.0, 4)          # z_0 = 0: every harmonic on row 0
    r = np.arange(16)
    assert np.allclose(S0[0], P[0, r] + P[0, 2 * r] + P[0, 3 * r] + P[0, 4 * r], rtol=0, atol=0)
    S3 = HS.harmonic_sum(P, 3.0, 0.0, 4)          # z_0 = 3: only the fundamental
    assert np.array_equal(S3[0], P[0, r])


def test_harmonic_series_of_chirps_sums_the_matched_powers():
    # noise-free complex chirps at (h r_bar, h z) with amplitudes a_h: each
    # sits on a grid cell with matched power a_h^2 N_t E_ret(h z) (the
    # injected-chirp pin of the plane), far apart in r, so the sum at the
    # fundamental's cell is the sum of those powers
    n_t, r_bar, z, m, H = 1 << 14, 1000, 2.0, 64, 4
    amps = [1.0, 0.7, 0.5, 0.3]
    x = np.zeros(n_t // 2, dtype=np.complex128)
    for h in range(1, H + 1):
        x += synth.complex_chirp_spectrum(n_t, h * r_bar - h * z / 2, h * z, amps[h - 1])
    zs = R.z_grid(-12.0, 2.0, 13)
    P = OP.plane(x.astype(np.complex64), R.template_taps(zs, m))
    S = HS.harmonic_sum(P, -12.0, 2.0, H)
    j = int(np.argmin(np.abs(zs - z)))
    e_ret = R.retained_energy([h * z for h in range(1, H + 1)], m)
    want = sum(amps[h - 1] ** 2 * n_t * e_ret[h - 1] for h in range(1, H + 1))
    assert abs(S[j, r_bar] / want - 1.0) < 2e-3
    # and the summed plane's maximum is that cell
    assert np.unravel_index(np.argmax(S), S.shape) == (j, r_bar)
