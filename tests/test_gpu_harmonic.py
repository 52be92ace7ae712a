"""GPU parity of the harmonic sum (fdas_harmonic_sum) with the oracle.

Both sides sum the same GPU plane (copied to the host), so the comparison
isolates the summing: FP64 planes must agree exactly (both add the harmonics
in order h = 1..H in double precision); FP32 sums within H 2^-23 relative
(sequential single-precision additions); BF16 outputs, rounded from single
precision, within one bfloat16 step of the oracle's double sum rounded the
same way.  Peaks of the summed plane must be the oracle's peaks of the oracle
sum; the peaks of sums that are never stored (fdas_harmonic_peaks) must be
bitwise the stored form's lists.  The full single-DM BF16 plane is checked on
sampled rows.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import harmonic as HS
from oracle import peaks as OK_PEAKS
from oracle import response as R

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def plan(dev, **kw):
    from paper_2206_12205_amd.fdas import Plan
    return Plan(device=dev, **kw)


def host(t):
    import torch
    return t.to(torch.float64).cpu().numpy()


def bf16_round(x):
    """Round float64 values to bfloat16 (nearest even) through float32, as float64."""
    import torch
    return torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def check(got, want, dtype, n_harm, what):
    assert got.shape == want.shape, what
    if dtype == "fp64":
        assert np.array_equal(got, want), what
    elif dtype == "fp32":
        err = np.abs(got - want) / np.maximum(np.abs(want), 1e-30)
        assert err.max() <= n_harm * 2.0 ** -23, f"{what}: {err.max():.3e}"
    else:
        w = bf16_round(want)
        # one bfloat16 step: 2^-7 of the value's binade
        step = np.exp2(np.floor(np.log2(np.maximum(np.abs(w), 1e-30))) - 7)
        d = np.abs(got - w)
        assert np.all(d <= step), f"{what}: {np.max(d / step):.2f} steps"
        assert np.mean(d != 0) < 0.01, what


C1 = synth.CONFIGS[1]


@pytest.mark.parametrize("pd", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("n_harm", [1, 2, 3, 8, 32])
def test_harmonic_sum_tiny_workload(dev, pd, n_harm):
    import torch
    say(f"[harmonic] tiny {pd} H={n_harm}")
    sp = synth.config1(0)
    compute = "fp64" if pd == "fp64" else "fp32"
    pl = plan(dev, max_bins=sp.spec.size, z_min=C1["z_min"], z_step=C1["z_step"], n_z=C1["n_z"],
              n_taps=C1["n_taps"], seg_len=C1["seg_len"], compute=compute, plane_dtype=pd)
    P = pl.correlate(torch.from_numpy(sp.spec).to(dev))
    S = pl.harmonic_sum(P, n_harm)
    want = HS.harmonic_sum(host(P), C1["z_min"], C1["z_step"], n_harm)
    check(host(S), want, pd, n_harm, f"{pd} H={n_harm}")


@pytest.mark.parametrize("z_min,z_step,n_z", [(-3.0, 2.0, 12), (0.0, 0.0, 1), (3.0, 0.0, 1), (-7.5, 1.25, 13)])
@pytest.mark.parametrize("n", [1, 5, 1023, 4097])
def test_harmonic_sum_grids_and_lengths(dev, z_min, z_step, n_z, n):
    """Grids with ties (h z_j halfway between rows), single templates with and
    without z = 0, lengths shorter than H and ragged block tails (FP64: exact)."""
    import torch
    say(f"[harmonic] grid z_min={z_min} step={z_step} n_z={n_z} n={n}")
    rng = np.random.default_rng(n + n_z)
    Ph = rng.exponential(size=(n_z, n))
    pl = plan(dev, max_bins=max(n, 2), z_min=z_min, z_step=z_step, n_z=n_z, n_taps=16, compute="fp64",
              plane_dtype="fp64")
    P = torch.from_numpy(Ph).to(dev)
    for H in (1, 2, 7, 32):
        S = pl.harmonic_sum(P, H)
        want = HS.harmonic_sum(Ph, z_min, z_step, H)
        assert np.array_equal(host(S), want), f"H={H}"


def test_peaks_of_the_summed_plane(dev):
    """fdas_peaks on the summed FP64 plane = the oracle's peaks of the oracle sum."""
    import torch
    say("[harmonic] peaks of the sum")
    sp = synth.config1(0)
    pl = plan(dev, max_bins=sp.spec.size, z_min=C1["z_min"], z_step=C1["z_step"], n_z=C1["n_z"],
              n_taps=C1["n_taps"], seg_len=C1["seg_len"], compute="fp64", plane_dtype="fp64")
    P = pl.correlate(torch.from_numpy(sp.spec).to(dev))
    for H in (2, 4):
        S = pl.harmonic_sum(P, H)
        want = HS.harmonic_sum(host(P), C1["z_min"], C1["z_step"], H)
        thr = 2.0 * H + 6.0
        got = pl.peaks(S, thr, capacity=4096)
        j, r, pw = OK_PEAKS.peaks(want, thr)
        assert got["n_found"] == len(j) > 0
        assert np.array_equal(got["z_idx"], j) and np.array_equal(got["r"], r)


@pytest.mark.parametrize("pd", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("n_harm", [1, 2, 8, 32])
def test_harmonic_sum_peaks_fused(dev, pd, n_harm):
    """fdas_harmonic_sum_peaks: the summed plane bitwise equal to
    fdas_harmonic_sum's, and exactly the oracle's peak list of that summed
    plane (thresholds above the noise, low, negative — every sum above — and
    NaN; a small capacity keeps the first entries and the true count)."""
    import torch
    say(f"[harmonic] fused sum+peaks {pd} H={n_harm}")
    sp = synth.config1(0)
    compute = "fp64" if pd == "fp64" else "fp32"
    pl = plan(dev, max_bins=sp.spec.size, z_min=C1["z_min"], z_step=C1["z_step"], n_z=C1["n_z"],
              n_taps=C1["n_taps"], seg_len=C1["seg_len"], compute=compute, plane_dtype=pd)
    P = pl.correlate(torch.from_numpy(sp.spec).to(dev))
    S = pl.harmonic_sum(P, n_harm)
    Sh = host(S)
    ints = {2: torch.int16, 4: torch.int32, 8: torch.int64}[S.element_size()]
    for thr, cap in ((2.0 * n_harm + 6.0, 4096), (3.0, 17), (-1.0, 1 << 20), (float("nan"), 8)):
        out = torch.full_like(S, float("nan"))
        S2, got = pl.harmonic_sum_peaks(P, n_harm, thr, capacity=cap, out=out, truncate=True)
        assert torch.equal(S2.view(ints), S.view(ints)), f"thr={thr}: summed plane differs"
        j, r, pw = OK_PEAKS.peaks(Sh, thr)
        k = min(len(j), cap)
        assert got["n_found"] == len(j), f"thr={thr}: {got['n_found']} vs {len(j)}"
        assert got["truncated"] == (len(j) > cap)
        assert np.array_equal(got["z_idx"], j[:k]) and np.array_equal(got["r"], r[:k]), f"thr={thr}"
        assert np.array_equal(got["power"].astype(np.float64), pw[:k].astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("pd", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("hs", [(2, 4, 8, 16), (1, 3, 32), (5,), (2, 3, 4, 5, 6, 7, 8, 9)])
def test_harmonic_sums_one_pass_equal_single_sums(dev, pd, hs):
    """fdas_harmonic_sums: every sum of the list bitwise equal to
    fdas_harmonic_sum's for the same H (the same additions in the same order),
    which the tests above hold against the oracle."""
    import torch
    say(f"[harmonic] one-pass sums {pd} {hs}")
    sp = synth.config1(0)
    compute = "fp64" if pd == "fp64" else "fp32"
    pl = plan(dev, max_bins=sp.spec.size, z_min=C1["z_min"], z_step=C1["z_step"], n_z=C1["n_z"],
              n_taps=C1["n_taps"], seg_len=C1["seg_len"], compute=compute, plane_dtype=pd)
    P = pl.correlate(torch.from_numpy(sp.spec).to(dev))
    got = pl.harmonic_sums(P, hs)
    ints = {2: torch.int16, 4: torch.int32, 8: torch.int64}[P.element_size()]
    for h, g in zip(hs, got):
        want = pl.harmonic_sum(P, h)
        assert torch.equal(g.view(ints), want.view(ints)), f"H={h}"


@pytest.mark.parametrize("pd", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("hs", [(2, 4, 8, 16), (1, 3, 32), (5,)])
def test_harmonic_sums_peaks_one_pass(dev, pd, hs):
    """fdas_harmonic_sums_peaks: the sums bitwise those of fdas_harmonic_sum,
    and each sum's list exactly the oracle's peaks of that sum (thresholds
    above the noise, low, negative and NaN across the levels)."""
    import torch
    say(f"[harmonic] one-pass sums with peaks {pd} {hs}")
    sp = synth.config1(0)
    compute = "fp64" if pd == "fp64" else "fp32"
    pl = plan(dev, max_bins=sp.spec.size, z_min=C1["z_min"], z_step=C1["z_step"], n_z=C1["n_z"],
              n_taps=C1["n_taps"], seg_len=C1["seg_len"], compute=compute, plane_dtype=pd)
    P = pl.correlate(torch.from_numpy(sp.spec).to(dev))
    ints = {2: torch.int16, 4: torch.int32, 8: torch.int64}[P.element_size()]
    for thrs in ([2.0 * h + 6.0 for h in hs], [3.0] * len(hs), [-1.0] + [float("nan")] * (len(hs) - 1)):
        sums, lists = pl.harmonic_sums_peaks(P, hs, thrs, capacity=1 << 20)
        for h, thr, S, got in zip(hs, thrs, sums, lists):
            want = pl.harmonic_sum(P, h)
            assert torch.equal(S.view(ints), want.view(ints)), f"H={h}"
            j, r, pw = OK_PEAKS.peaks(host(want), thr)
            assert got["n_found"] == len(j), f"H={h} thr={thr}: {got['n_found']} vs {len(j)}"
            assert np.array_equal(got["z_idx"], j) and np.array_equal(got["r"], r), f"H={h} thr={thr}"


@pytest.mark.parametrize("pd", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("hs", [(2, 4, 8, 16), (1, 3, 32), (5,)])
def test_harmonic_peaks_unstored_equal_stored(dev, pd, hs):
    """fdas_harmonic_peaks (the sums never stored, flagged tiles recomputed
    from the plane): every list bitwise fdas_harmonic_sums_peaks's (cells,
    order, powers, true count) and the oracle's peaks of the summed plane, at
    thresholds above the noise, low with a small capacity (the first entries
    and the true count), negative and NaN; a length with a ragged last tile."""
    import torch
    say(f"[harmonic] peaks of unstored sums {pd} {hs}")
    sp = synth.config1(0)
    n = sp.spec.size - 37
    compute = "fp64" if pd == "fp64" else "fp32"
    pl = plan(dev, max_bins=sp.spec.size, z_min=C1["z_min"], z_step=C1["z_step"], n_z=C1["n_z"],
              n_taps=C1["n_taps"], seg_len=C1["seg_len"], compute=compute, plane_dtype=pd)
    P = pl.correlate(torch.from_numpy(sp.spec[:n]).to(dev))
    for thrs, cap in (([2.0 * h + 6.0 for h in hs], 1 << 20), ([3.0] * len(hs), 17),
                      ([-1.0] + [float("nan")] * (len(hs) - 1), 1 << 20)):
        _, want = pl.harmonic_sums_peaks(P, hs, thrs, capacity=cap, truncate=True)
        got = pl.harmonic_peaks(P, hs, thrs, capacity=cap, truncate=True)
        for h, thr, a, b in zip(hs, thrs, got, want):
            what = f"H={h} thr={thr} cap={cap}"
            assert a["n_found"] == b["n_found"], what
            for k in ("z_idx", "r", "power"):
                assert np.array_equal(a[k], b[k]), f"{what} {k}"
            if cap > 1 << 16:
                j, r, _ = OK_PEAKS.peaks(host(pl.harmonic_sum(P, h)), thr)
                assert a["n_found"] == len(j) and np.array_equal(a["z_idx"], j) and np.array_equal(a["r"], r), what


def test_harmonic_series_of_chirps_on_the_gpu(dev):
    """The sum at the fundamental's cell of a noise-free harmonic series of
    chirps is the sum of their matched powers (the oracle pin's physics),
    through the GPU plane and the GPU sum."""
    import torch
    say("[harmonic] chirp series")
    n_t, r_bar, z, m, H = 1 << 14, 1000, 2.0, 64, 4
    amps = [1.0, 0.7, 0.5, 0.3]
    x = np.zeros(n_t // 2, dtype=np.complex128)
    for h in range(1, H + 1):
        x += synth.complex_chirp_spectrum(n_t, h * r_bar - h * z / 2, h * z, amps[h - 1])
    pl = plan(dev, max_bins=x.size, z_min=-12.0, z_step=2.0, n_z=13, n_taps=m, seg_len=1024, compute="fp32")
    S = host(pl.harmonic_sum(pl.correlate(torch.from_numpy(x.astype(np.complex64)).to(dev)), H))
    e_ret = R.retained_energy([h * z for h in range(1, H + 1)], m)
    want = sum(amps[h - 1] ** 2 * n_t * e_ret[h - 1] for h in range(1, H + 1))
    j = 7                                                   # z = 2 on the grid -12, -10, ..., 12
    assert np.unravel_index(np.argmax(S), S.shape) == (j, r_bar)
    assert abs(S[j, r_bar] / want - 1.0) < 2e-3


def test_single_dm_bf16_plane_sampled_rows(dev):
    """Full single-DM size (101 x 4,194,304 BF16 plane, H = 8): the GPU sum on
    sampled output rows (both ends, the z = 0 row and rows whose harmonics run
    off the grid) against the oracle's sum of the same plane."""
    import torch
    c = synth.CONFIGS[2]
    say("[harmonic] single-DM bf16 H=8")
    x, _ = synth.config2_device(dev, 0)
    n = x.numel()
    pl = plan(dev, max_bins=n, z_min=c["z_min"], z_step=c["z_step"], n_z=c["n_z"], n_taps=c["n_taps"],
              compute="bf16", plane_dtype="bf16")
    P = pl.correlate(x)
    S = pl.harmonic_sum(P, 8)
    torch.cuda.synchronize()
    Ph = P.view(torch.int16).cpu().numpy().view(np.uint16)    # raw bfloat16
    Pf = (Ph.astype(np.uint32) << 16).view(np.float32)        # exact widening
    rows = [0, 3, 44, 49, 50, 51, 56, 57, 100]
    want = HS.harmonic_sum(Pf, c["z_min"], c["z_step"], 8, out_rows=rows)
    got = host(S[rows])
    check(got, want, "bf16", 8, "single-DM rows")
    # the fused call at full size: the same summed plane and the list
    # fdas_peaks gives for it
    for thr in (c["threshold"], 20.0):
        a = pl.peaks(S, thr, capacity=1 << 20)
        S2, b = pl.harmonic_sum_peaks(P, 8, thr, capacity=1 << 20)
        assert torch.equal(S2.view(torch.int16), S.view(torch.int16))
        assert a["n_found"] == b["n_found"]
        assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["z_idx"], b["z_idx"])
    # several sums in one pass at full size: each bitwise the single-H sum
    sums = pl.harmonic_sums(P, (2, 4, 8, 16))
    for h, g in zip((2, 4, 8, 16), sums):
        assert torch.equal(g.view(torch.int16), pl.harmonic_sum(P, h).view(torch.int16)), f"H={h}"
    sums, lists = pl.harmonic_sums_peaks(P, (2, 4, 8, 16), [c["threshold"] + 10.0 * k for k in (1, 2, 3, 4)],
                                         capacity=1 << 20)
    for h, S, got, thr in zip((2, 4, 8, 16), sums, lists, [c["threshold"] + 10.0 * k for k in (1, 2, 3, 4)]):
        ref = pl.peaks(pl.harmonic_sum(P, h), thr, capacity=1 << 20)
        assert got["n_found"] == ref["n_found"] and np.array_equal(got["r"], ref["r"]), f"H={h}"


@pytest.mark.parametrize("pd", ["fp32", "bf16", "fp64"])
def test_harmonic_marks_survive_nan_sums(dev, pd):
    """NaN cells in the plane: a thread whose sums in one peak tile are
    (above the threshold, NaN, below, below) must still flag the tile, so
    the fused calls (and the unstored form) list exactly the oracle's peaks of
    the summed plane.
    Each thread holds the fundamentals r0 + 256 i, four per 1024-bin tile."""
    import torch
    say(f"[harmonic] NaN sums beside peaks {pd}")
    n_z, n = 5, 16384
    compute = "fp64" if pd == "fp64" else "fp32"
    pl = plan(dev, max_bins=n, z_min=-4.0, z_step=2.0, n_z=n_z, n_taps=64, seg_len=1024, compute=compute,
              plane_dtype=pd)
    g = np.random.default_rng(5)
    base = g.uniform(0.0, 1.0, size=(n_z, n))
    tdt = {"fp32": torch.float32, "bf16": torch.bfloat16, "fp64": torch.float64}[pd]
    for H in (1, 3):
        nh = (n - 1) // H + 1
        Pn = base.copy()
        cells = [(1, 100), (3, 1024 + 37), (2, 4096 + 700)]    # fundamentals in three tiles
        for j, r in cells:
            # row j of the sum is row j of the plane for z = 0 rows only; put
            # the bright term on every row the harmonics of (j, r) read
            for h in range(1, H + 1):
                Pn[:, h * r] = 0.0
            Pn[j, r] = 60.0
            Pn[:, r + 256] = np.nan              # the same thread's next sum in that tile
        P = torch.from_numpy(Pn).to(tdt).to(dev).contiguous()
        S = pl.harmonic_sum(P, H)
        Sh = host(S)
        thr = 50.0
        j, r, _ = OK_PEAKS.peaks(Sh, thr)
        assert len(j) >= len(cells)
        _, got = pl.harmonic_sum_peaks(P, H, thr, capacity=1 << 12)
        assert np.array_equal(got["z_idx"], j) and np.array_equal(got["r"], r), f"H={H} single"
        _, lists = pl.harmonic_sums_peaks(P, [H], [thr], capacity=1 << 12)
        assert np.array_equal(lists[0]["z_idx"], j) and np.array_equal(lists[0]["r"], r), f"H={H} one-pass"
        unstored = pl.harmonic_peaks(P, [H], [thr], capacity=1 << 12)
        assert np.array_equal(unstored[0]["z_idx"], j) and np.array_equal(unstored[0]["r"], r), f"H={H} unstored"
        assert nh == S.shape[1]
