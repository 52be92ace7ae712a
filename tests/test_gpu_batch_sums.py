"""GPU checks of fdas_batch_harmonic_sums_peaks: the harmonic sums of every
job of a batch with their thresholded peaks, the sums never stored.

Bars (integer and index work on the same planes): every (level, job) list
is bitwise the list fdas_harmonic_sums_peaks gives for that job's plane (the
same cells in the same order, the same powers, the same true count), and the
oracle's peak definition applied to the oracle's sum of the GPU plane
(oracle/harmonic.py, rounded to the plane type as the stored sum is) gives the
same cells.  Ragged jobs (1 .. 200,000 bins), BF16 / FP32 / FP64 planes,
thresholds with few peaks, many peaks (small capacity: the first entries and
the true count) and none; lengths in whole 16-byte chunks beside ragged
ones; z grids symmetric about z = 0, offset, one-sided and of 201 templates.
"""
import sys

import numpy as np
import pytest

from oracle import harmonic as HS
from oracle import peaks as OK_PEAKS

pytestmark = pytest.mark.gpu

ZMIN, ZSTEP, NZ, M = -16.0, 2.0, 17, 128
# ragged lengths, and lengths in whole 16-byte chunks of every plane type
LENGTHS = [70001, 1, 3839, 12345, 200000, 517, 1025, 40000]
CHUNKED = [70000, 8, 3840, 12344, 200000, 520, 1024, 40000]
REC = np.dtype([("r", "<i8"), ("z_idx", "<i4"), ("job", "<i4"), ("power", "<f4"), ("reserved", "<f4")])


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def noise_planes(dev, pl, seed, dtype):
    """Exp(1) noise planes for the stored batch with a few bright cells."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    P = -torch.log1p(-torch.rand(pl.batch_cells, generator=g, dtype=torch.float64))
    idx = torch.randint(0, pl.batch_cells, (60,), generator=g)
    P[idx] = 20.0 + 40.0 * torch.rand(60, generator=g, dtype=torch.float64)
    return P.to(dtype).to(dev).contiguous()


@pytest.mark.parametrize("form", ["ragged", "chunked"])
@pytest.mark.parametrize("plane_dtype", ["bf16", "fp32", "fp64"])
def test_batch_sums_match_per_job_calls(dev, plane_dtype, form):
    import torch
    from paper_2206_12205_amd.fdas import Plan
    tdt = {"bf16": torch.bfloat16, "fp32": torch.float32, "fp64": torch.float64}[plane_dtype]
    compute = "fp64" if plane_dtype == "fp64" else "fp32"
    lengths = LENGTHS if form == "ragged" else CHUNKED
    pl = Plan(max_bins=max(lengths), z_min=ZMIN, z_step=ZSTEP, n_z=NZ, n_taps=M, compute=compute,
              plane_dtype=plane_dtype, device=dev, max_jobs=len(lengths))
    pl.set_batch(lengths)
    planes = noise_planes(dev, pl, 7, tdt)
    hs = [2, 4, 8, 16]
    cases = (([12.0, 16.0, 24.0, 36.0], 1 << 14), ([6.0, 9.0, 14.0, 24.0], 40), ([1e9] * 4, 4))
    for thr, cap in cases:
        say(f"[batch sums] {plane_dtype} thresholds {thr} capacity {cap}")
        got = pl.batch_sums_peaks(planes, hs, thr, capacity=cap, truncate=True)
        for i, n in enumerate(lengths):
            P = pl.batch_plane(planes, i).contiguous()
            _, want = pl.harmonic_sums_peaks(P, hs, thr, capacity=cap, truncate=True)
            for l, h in enumerate(hs):
                a, b = got[l][i], want[l]
                what = f"{form} job {i} (n={n}) H={h}"
                assert a["n_found"] == b["n_found"], what
                assert np.array_equal(a["z_idx"], b["z_idx"]) and np.array_equal(a["r"], b["r"]), what
                assert np.array_equal(a["power"], b["power"]), what
                assert np.all(a["job"] == i), what
        # the oracle on the two longest jobs at the first thresholds
        if cap == 1 << 14:
            for i in (4, 0):
                host = pl.batch_plane(planes, i).to(torch.float64).cpu().numpy()
                for l, h in enumerate(hs):
                    S = HS.harmonic_sum(host, ZMIN, ZSTEP, h)
                    if plane_dtype == "bf16":
                        S = torch.from_numpy(S.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
                    elif plane_dtype == "fp32":
                        S = S.astype(np.float32).astype(np.float64)
                    j, r, _ = OK_PEAKS.peaks(S, thr[l])
                    a = got[l][i]
                    # the GPU adds in single precision (BF16 / FP32 planes), the
                    # oracle in double: compare the cells whose margins clear
                    # that rounding (one bfloat16 step for BF16 sums)
                    tol = {"bf16": 1e-2, "fp32": 1e-5, "fp64": 1e-9}[plane_dtype]
                    amb = OK_PEAKS.margins(S, j, r, thr[l]) < tol
                    oset = {x for x, m in zip(zip(j.tolist(), r.tolist()), amb) if not m}
                    gset = set(zip(a["z_idx"].tolist(), a["r"].tolist()))
                    assert oset <= gset, f"job {i} H={h}: {sorted(oset - gset)[:5]}"


def test_batch_sums_single_harmonic_is_the_plane(dev):
    """H = 1 is the plane itself (one term, added to zero, rounded as stored):
    its list for every job equals fdas_peaks of that job's plane, beside a
    second level H = 3 checked against the per-job call."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    pl = Plan(max_bins=max(LENGTHS), z_min=ZMIN, z_step=ZSTEP, n_z=NZ, n_taps=M, compute="bf16",
              plane_dtype="bf16", device=dev, max_jobs=len(LENGTHS))
    pl.set_batch(LENGTHS)
    planes = noise_planes(dev, pl, 11, torch.bfloat16)
    hs, thr = [1, 3], [7.0, 12.0]
    got = pl.batch_sums_peaks(planes, hs, thr, capacity=1 << 14, truncate=True)
    for i, n in enumerate(LENGTHS):
        P = pl.batch_plane(planes, i).contiguous()
        want1 = pl.peaks(P, thr[0], capacity=1 << 14, truncate=True)
        _, want = pl.harmonic_sums_peaks(P, hs, thr, capacity=1 << 14, truncate=True)
        for a, b, what in ((got[0][i], want1, "H=1 vs fdas_peaks"), (got[1][i], want[1], "H=3")):
            assert a["n_found"] == b["n_found"], f"job {i} {what}"
            for k in ("z_idx", "r", "power"):
                assert np.array_equal(a[k], b[k]), f"job {i} {what} {k}"
        assert got[0][i]["n_found"] > 0 or n < 100


def test_batch_sums_on_an_unaligned_grid(dev):
    """A z grid whose z_min is no multiple of z_step (the workgroup order's
    template families do not exist there): the lists still equal the
    per-job calls."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    pl = Plan(max_bins=max(LENGTHS), z_min=-15.0, z_step=1.7, n_z=19, n_taps=M, compute="fp32",
              plane_dtype="fp32", device=dev, max_jobs=len(LENGTHS))
    pl.set_batch(LENGTHS)
    planes = noise_planes(dev, pl, 13, torch.float32)
    hs, thr = [2, 5, 9], [10.0, 18.0, 27.0]
    got = pl.batch_sums_peaks(planes, hs, thr, capacity=1 << 14, truncate=True)
    for i, n in enumerate(LENGTHS):
        P = pl.batch_plane(planes, i).contiguous()
        _, want = pl.harmonic_sums_peaks(P, hs, thr, capacity=1 << 14, truncate=True)
        for l, h in enumerate(hs):
            a, b = got[l][i], want[l]
            assert a["n_found"] == b["n_found"], f"job {i} H={h}"
            for k in ("z_idx", "r", "power"):
                assert np.array_equal(a[k], b[k]), f"job {i} H={h} {k}"


def _per_job_lists_equal(pl, planes, lengths, hs, thr, cap, what):
    got = pl.batch_sums_peaks(planes, hs, thr, capacity=cap, truncate=True)
    total = 0
    for i, n in enumerate(lengths):
        P = pl.batch_plane(planes, i).contiguous()
        _, want = pl.harmonic_sums_peaks(P, hs, thr, capacity=cap, truncate=True)
        for l, h in enumerate(hs):
            a, b = got[l][i], want[l]
            assert a["n_found"] == b["n_found"], f"{what} job {i} (n={n}) H={h}"
            for k in ("z_idx", "r", "power"):
                assert np.array_equal(a[k], b[k]), f"{what} job {i} (n={n}) H={h} {k}"
            total += int(a["n_found"])
    return total


@pytest.mark.parametrize("z_min,z_step,n_z", [
    (-100.0, 2.0, 101),   # the single-DM grid: 50 rows each side and z = 0
    (-10.0, 1.0, 60),     # values -10 .. 49: sides of different sizes
    (10.0, 1.0, 60),      # values 10 .. 69: positive rows only, none below 10
    (-40.0, 1.0, 30),     # values -40 .. -11: negative rows only
    (-200.0, 2.0, 201),   # 201 templates
])
def test_batch_sums_on_other_grids(dev, z_min, z_step, n_z):
    """Grids beside the default one (template families reach the grid edge
    at other harmonics, or exist on one side only): every (level, job) list
    equals the per-job call's, at thresholds with many peaks."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    lengths = [65536, 8, 4104, 24576, 131072, 1000] if n_z <= 101 else [16384, 4096, 1000]
    pl = Plan(max_bins=max(lengths), z_min=z_min, z_step=z_step, n_z=n_z, n_taps=M, compute="bf16",
              plane_dtype="bf16", device=dev, max_jobs=len(lengths))
    pl.set_batch(lengths)
    planes = noise_planes(dev, pl, 17, torch.bfloat16)
    hs, thr = [2, 3, 8, 16, 32], [9.0, 12.0, 20.0, 32.0, 52.0]
    say(f"[batch sums] grid {z_min} {z_step} {n_z}")
    total = _per_job_lists_equal(pl, planes, lengths, hs, thr, 1 << 15, f"grid {z_min}/{z_step}/{n_z}")
    assert total > 100
