"""GPU checks of peak finding fused with the plane store
(fdas_correlate_peaks, fdas_correlate_batch_peaks).

Bars.  The fused plane is bitwise the plane fdas_correlate writes (the same
kernel arithmetic; marking only adds flag stores).  Peak lists are integer
and index work on that plane, so they are held bit-exactly against the
oracle's peak definition (oracle/peaks.py) applied to the GPU plane: the same
(z_idx, r) list in order, the same powers, the true count, and with a small
capacity the first `capacity` entries.  Batched: job i's list is the
oracle's list of job i's plane, with job = i.  Thresholds cover the common
case (few tiles above), a low one (most tiles above), a negative one (every
cell above: the prefilter must pass everything) and NaN (nothing above).
At the single-DM size the fused list must equal fdas_peaks's on the same
plane, and every listed peak is checked against its 3x3 neighbourhood with
the oracle's margins.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import peaks as OK_PEAKS

pytestmark = pytest.mark.gpu

ZMIN, ZSTEP, NZ, M = -16.0, 2.0, 17, 256


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(spec, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(spec, dtype=np.complex64)).to(dev)


def widen(plane):
    import torch
    return plane.to(torch.float64).cpu().numpy()


def spectrum(n, seed):
    """Seeded noise spectrum with a few chirps (bright peaks on some rows)."""
    x = synth.random_spectrum(n, seed).astype(np.complex128)
    g = np.random.default_rng(seed + 1)
    for _ in range(3):
        if n < 64:
            break
        r0 = float(g.uniform(16, n - 16))
        z = float(g.uniform(ZMIN, -ZMIN))
        k = np.arange(n)
        q = k - r0
        x += 3.0 * np.exp(-0.5 * (q / 2.0) ** 2) * np.exp(1j * math.pi * z * (q / max(n, 1)) ** 2)
    return x


def assert_same_peaks(got, host, thr, cap, job=None, what=""):
    j, r, pw = OK_PEAKS.peaks(host, thr)
    assert got["n_found"] == len(j), f"{what}: count {got['n_found']} vs {len(j)}"
    k = min(len(j), cap)
    assert np.array_equal(got["z_idx"], j[:k]), what
    assert np.array_equal(got["r"], r[:k]), what
    assert np.array_equal(got["power"].astype(np.float64), pw[:k]), what
    if job is not None:
        assert np.all(got["job"] == job), what


PLANS = [
    dict(compute="bf16", plane_dtype="bf16"),                 # matrix-core L = 4096: marks in the kernel
    dict(compute="bf16", plane_dtype="fp32"),                 # same kernel, FP32 plane
    dict(compute="fp32", plane_dtype="fp32"),                 # vector-ALU kernel: separate mark pass
    dict(compute="bf16", plane_dtype="bf16", algo="valu"),
]


@pytest.mark.parametrize("kw", PLANS, ids=lambda k: "-".join(str(v) for v in k.values()))
@pytest.mark.parametrize("n", [1, 7, 3841, 17 * 1024 + 5, 200003])
def test_fused_single_matches_oracle(dev, kw, n):
    import torch
    from paper_2206_12205_amd.fdas import Plan
    say(f"[fused] single {kw} n={n}")
    pl = Plan(max_bins=200003, z_min=ZMIN, z_step=ZSTEP, n_z=NZ, n_taps=M, device=dev, **kw)
    x = to_dev(spectrum(n, 11 + n), dev)
    ref = pl.correlate(x)
    host = widen(ref)
    for thr, cap in ((12.0, 1 << 16), (3.0, 1 << 18), (3.0, 7), (-1.0, 1 << 22), (float("nan"), 16)):
        plane = torch.full_like(ref, float("nan"))
        plane, got = pl.correlate_peaks(x, thr, capacity=cap, plane=plane, truncate=True)
        assert torch.equal(plane.view(torch.int16 if plane.element_size() == 2 else torch.int32),
                           ref.view(torch.int16 if ref.element_size() == 2 else torch.int32)), "plane differs"
        assert_same_peaks(got, host, thr, cap, job=0, what=f"thr={thr} cap={cap}")
    # the fused list equals fdas_peaks on the same plane
    a = pl.peaks(ref, 3.0, capacity=1 << 18)
    _, b = pl.correlate_peaks(x, 3.0, capacity=1 << 18)
    assert a["n_found"] == b["n_found"] and np.array_equal(a["r"], b["r"]) and np.array_equal(a["z_idx"], b["z_idx"])


LENGTHS = [70001, 1, 3839, 3840, 3841, 12345, 200000, 517, 1024, 1025]


@pytest.mark.parametrize("kw", [PLANS[0], PLANS[1], PLANS[2]], ids=["m4k-bf16", "m4k-fp32", "valu-fp32"])
def test_fused_batch_matches_oracle(dev, kw):
    import torch
    from paper_2206_12205_amd.fdas import Plan
    say(f"[fused] batch {kw}")
    pl = Plan(max_bins=max(LENGTHS), z_min=ZMIN, z_step=ZSTEP, n_z=NZ, n_taps=M, device=dev,
              max_jobs=len(LENGTHS), **kw)
    pl.set_batch(LENGTHS)
    spectra = torch.cat([to_dev(spectrum(v, 100 + i), dev) for i, v in enumerate(LENGTHS)])
    ref = pl.correlate_batch(spectra)
    for thr, cap in ((12.0, 1 << 14), (3.0, 33), (-1.0, 1 << 22), (float("nan"), 4)):
        planes = torch.full_like(ref, float("nan"))
        planes, got = pl.correlate_batch_peaks(spectra, thr, capacity=cap, planes=planes, truncate=True)
        assert torch.equal(planes.view(torch.int16 if planes.element_size() == 2 else torch.int32),
                           ref.view(torch.int16 if ref.element_size() == 2 else torch.int32)), "planes differ"
        for i in range(len(LENGTHS)):
            host = widen(pl.batch_plane(ref, i))
            assert_same_peaks(got[i], host, thr, cap, job=i, what=f"job {i} thr={thr} cap={cap}")


@pytest.mark.parametrize("pd", ["bf16", "fp32"])
@pytest.mark.parametrize("taps", [2, 130])
def test_fused_rows_anywhere_small_and_odd_taps(dev, taps, pd):
    """Matrix-core planes (BF16 and FP32) whose rows start anywhere, with 2 taps (the
    kept samples reach the segment's last run) and 130 (an odd half-width):
    single calls and one batch, plain and fused.  The batch's planes are
    bitwise the single calls', the fused planes bitwise the plain ones, and
    every list is the oracle's on its plane."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    lengths = [9001, 12347, 3 * 4096 + 5, 20002, 7]
    kw = dict(z_min=ZMIN, z_step=ZSTEP, n_z=NZ, n_taps=taps, seg_len=4096, compute="bf16",
              plane_dtype=pd, algo="mfma", device=dev)
    it = torch.int16 if pd == "bf16" else torch.int32
    pl = Plan(max_bins=max(lengths), max_jobs=len(lengths), **kw)
    specs = [to_dev(spectrum(v, 700 + taps + i), dev) for i, v in enumerate(lengths)]
    singles = []
    for i, x in enumerate(specs):
        say(f"[fused] rows anywhere taps={taps} {pd} single n={lengths[i]}")
        ref = pl.correlate(x)
        singles.append(ref)
        for thr, cap in ((12.0, 1 << 14), (-1.0, 1 << 20)):
            plane, got = pl.correlate_peaks(x, thr, capacity=cap, truncate=True)
            assert torch.equal(plane.view(it), ref.view(it)), f"n={lengths[i]} fused plane"
            assert_same_peaks(got, widen(ref), thr, cap, what=f"single n={lengths[i]} thr={thr}")
    say(f"[fused] rows anywhere taps={taps} {pd} batch")
    pl.set_batch(lengths)
    spectra = torch.cat(specs)
    planes = pl.correlate_batch(spectra)
    for i in range(len(lengths)):
        assert torch.equal(pl.batch_plane(planes, i).view(it), singles[i].view(it)), \
            f"batch job {i} differs from its single call"
    for thr, cap in ((12.0, 1 << 14), (-1.0, 1 << 20)):
        fused, got = pl.correlate_batch_peaks(spectra, thr, capacity=cap, truncate=True)
        assert torch.equal(fused.view(it), planes.view(it)), "fused batch planes"
        for i in range(len(lengths)):
            assert_same_peaks(got[i], widen(singles[i]), thr, cap, job=i, what=f"batch job {i} thr={thr}")


def test_fused_batch_graph_replays(dev):
    """One fdas_correlate_batch_peaks recorded as a HIP graph, replayed on new
    spectra with eager work between replays; every replay equals the eager
    call."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    say("[fused] batch graph")
    lengths = [50000, 3841, 9, 123457]
    pl = Plan(max_bins=max(lengths), z_min=ZMIN, z_step=ZSTEP, n_z=NZ, n_taps=M, device=dev,
              max_jobs=len(lengths), compute="bf16", plane_dtype="bf16")
    pl.set_batch(lengths)
    cap = 1 << 12
    spectra = torch.cat([to_dev(spectrum(v, 300 + i), dev) for i, v in enumerate(lengths)])
    planes = torch.empty(pl.batch_cells, dtype=torch.bfloat16, device=dev)
    out = torch.zeros((len(lengths), cap, 24), dtype=torch.uint8, device=dev)
    nf = torch.zeros(len(lengths), dtype=torch.int64, device=dev)
    pl.batch_peaks_scratch()                      # allocated before capture
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        pl.correlate_batch_peaks_async(spectra, planes, 5.0, out, nf)
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize(dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pl.correlate_batch_peaks_async(spectra, planes, 5.0, out, nf)
    for rep in range(3):
        fresh = torch.cat([to_dev(spectrum(v, 400 + 10 * rep + i), dev) for i, v in enumerate(lengths)])
        spectra.copy_(fresh)
        planes.fill_(0)
        out.zero_()
        nf.fill_(-1)
        torch.cuda.synchronize(dev)
        g.replay()
        torch.cuda.synchronize(dev)
        _, want = pl.correlate_batch_peaks(fresh, 5.0, capacity=cap, truncate=True)
        found = nf.cpu().tolist()
        for i in range(len(lengths)):
            assert found[i] == want[i]["n_found"], f"replay {rep} job {i}"
            k = min(found[i], cap)
            rec = out[i, :k].cpu().numpy().view(np.dtype([("r", "<i8"), ("z_idx", "<i4"), ("job", "<i4"),
                                                          ("power", "<f4"), ("reserved", "<f4")])).reshape(-1)
            assert np.array_equal(rec["r"], want[i]["r"]) and np.array_equal(rec["z_idx"], want[i]["z_idx"])
            assert np.all(rec["job"] == i)


def test_fused_single_dm_full_size(dev):
    """The single-DM workload at full size (4,194,304 bins x 101 templates,
    BF16, the benchmark's plan): the fused list equals fdas_peaks's on the
    same plane, and every listed peak passes the oracle's 3x3 test."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    c = synth.CONFIGS[2]
    say("[fused] single-DM full size")
    sp = synth.config2(6)                                   # a bright pulsar (P1 ~ 3000)
    x = to_dev(sp.spec, dev)
    pl = Plan(max_bins=sp.spec.size, z_min=c["z_min"], z_step=c["z_step"], n_z=c["n_z"], n_taps=c["n_taps"],
              compute="bf16", plane_dtype="bf16", device=dev)
    ref = pl.correlate(x)
    for thr in (c["threshold"], 12.0):                      # the workload's threshold, and noise peaks
        a = pl.peaks(ref, thr, capacity=1 << 20)
        plane, b = pl.correlate_peaks(x, thr, capacity=1 << 20)
        assert torch.equal(plane.view(torch.int16), ref.view(torch.int16))
        assert a["n_found"] == b["n_found"] and a["n_found"] > 0
        assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["z_idx"], b["z_idx"])
        assert np.array_equal(a["power"], b["power"])
        # every listed peak (a sample of up to ~2000): above the threshold
        # and a 3x3 local maximum
        sample = np.arange(len(b["r"]))[:: max(1, len(b["r"]) // 2000)]
        for i in sample:
            j, r = int(b["z_idx"][i]), int(b["r"][i])
            lo, hi = max(j - 1, 0), min(j + 2, c["n_z"])
            a0, a1 = max(r - 1, 0), min(r + 2, sp.spec.size)
            win = widen(ref[lo:hi, a0:a1])
            P = np.full((3, 3), -np.inf)
            P[lo - j + 1:hi - j + 1, a0 - r + 1:a1 - r + 1] = win
            jj, rr, _ = OK_PEAKS.peaks(P, thr)
            assert (1, 1) in set(zip(jj.tolist(), rr.tolist())), f"peak {i} at ({j}, {r})"
