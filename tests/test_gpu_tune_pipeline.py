"""GPU checks of the autotuner (fdas_tune) and of the batched search over
many spectra (length classes, tuned plans, chunked plane buffer, peaks)."""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import peaks as OPK
from oracle import plane as OP
from oracle import response as R

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


C1 = synth.CONFIGS[1]


@pytest.mark.parametrize("compute", ["fp32", "bf16"])
def test_tune_picks_a_valid_configuration(dev, compute):
    import torch
    from paper_2206_12205_amd.fdas import Plan, tune
    say(f"[tune] {compute}")
    sp = synth.config1(0)
    x = torch.from_numpy(sp.spec).to(dev)
    t = tune(x, C1["z_min"], C1["z_step"], C1["n_z"], C1["n_taps"], compute=compute, reps=3)
    say(f"  -> {t}")
    assert t["ms"] > 0 and 1 <= t["z_chunk"] <= C1["n_z"]
    assert t["seg_len"] in (1024, 2048, 4096, 8192, 16384)
    assert compute == "bf16" or t["algo"] == "valu"
    # a fixed knob is kept
    t2 = tune(x, C1["z_min"], C1["z_step"], C1["n_z"], C1["n_taps"], compute=compute, seg_len=2048, reps=2)
    assert t2["seg_len"] == 2048 and t2["algo"] == "valu"
    # the chosen plan computes the plane (oracle bars of the precision form)
    pl = Plan(x.numel(), C1["z_min"], C1["z_step"], C1["n_z"], C1["n_taps"], t["seg_len"], compute=compute,
              algo=t["algo"], z_chunk=t["z_chunk"], device=dev)
    p = pl.correlate(x).double().cpu().numpy()[:, 1000:1400]
    taps = R.template_taps(R.z_grid(C1["z_min"], C1["z_step"], C1["n_z"]), C1["n_taps"])
    ref = OP.plane(sp.spec, taps, 1000, 1400)
    err = np.abs(p - ref) / np.maximum(ref, 1.0)
    assert err.max() <= (1e-4 if compute == "fp32" else 0.15)


def batch_spectra(lengths, seed):
    """Unit-power complex noise per job plus one bright complex chirp in every
    other job (so the peak lists are not empty)."""
    g = np.random.default_rng(seed)
    parts = []
    for i, n in enumerate(lengths):
        x = synth.random_spectrum(n, seed=seed * 1000 + i).astype(np.complex128)
        if i % 2 == 0 and n > 600:
            r_bar = float(g.uniform(200, n - 200))
            z = float(g.uniform(-12, 12))
            x[:] += synth.complex_chirp_spectrum(2 * n, r_bar - z / 2, z, amp=0.25)[:n]
        parts.append(x.astype(np.complex64))
    return parts


def test_batch_search_matches_single_plans(dev):
    import torch
    from paper_2206_12205_amd.fdas import Plan
    from paper_2206_12205_amd.pipeline import BatchSearch
    lengths = [20000, 70001, 3001, 150000, 9000, 40000, 1, 131072]
    n_z, M = 9, 128
    say(f"[pipeline] lengths {lengths}")
    parts = batch_spectra(lengths, seed=11)
    x = torch.from_numpy(np.concatenate(parts)).to(dev)
    # a buffer of about two of the longest planes forces several chunks
    bs = BatchSearch(lengths, -8.0, 2.0, n_z, M, compute="bf16", plane_dtype="bf16",
                     buffer_bytes=n_z * 160000 * 2 * 2, device=dev, peak_capacity=256)
    assert len(bs.chunks) >= 3
    thr = 20.0
    bs.run(x, thr)
    torch.cuda.synchronize()
    for cls, t in bs.tuned.items():
        say(f"  class 2^{cls}: {t}")
    for i, n in enumerate(lengths):
        cls = max(int(math.ceil(math.log2(n))), 0)
        t = bs.tuned[cls]
        cmax = max(v for v in lengths if max(int(math.ceil(math.log2(v))), 0) == cls)
        pl = Plan(cmax, -8.0, 2.0, n_z, M, t["seg_len"], compute="bf16", plane_dtype="bf16", algo=t["algo"],
                  z_chunk=t["z_chunk"], device=dev)
        xi = torch.from_numpy(parts[i]).to(dev)
        ref = pl.peaks(pl.correlate(xi), thr, capacity=256)
        got = bs.peaks(i)
        assert got["n_found"] == ref["n_found"], f"job {i}"
        for k in ("z_idx", "r", "power"):
            assert np.array_equal(got[k], ref[k]), f"job {i} {k}"
        if i % 2 == 0 and n > 600:
            assert got["n_found"] >= 1


def test_batch_search_strong_peak_vs_oracle(dev):
    """The brightest peak of a chirp job sits where the oracle plane's maximum is."""
    import torch
    from paper_2206_12205_amd.pipeline import BatchSearch
    lengths = [30000, 5000]
    n_z, M = 9, 128
    parts = batch_spectra(lengths, seed=12)
    x = torch.from_numpy(np.concatenate(parts)).to(dev)
    bs = BatchSearch(lengths, -8.0, 2.0, n_z, M, device=dev, peak_capacity=1024)
    bs.run(x, 20.0)
    torch.cuda.synchronize()
    got = bs.peaks(0)
    k = int(np.argmax(got["power"]))
    taps = R.template_taps(R.z_grid(-8.0, 2.0, n_z), M)
    ref = OP.plane(parts[0], taps)
    jz, jr = np.unravel_index(np.argmax(ref), ref.shape)
    assert (got["z_idx"][k], got["r"][k]) == (jz, jr)
    _, ro_r, _ = OPK.peaks(ref, 20.0)
    assert abs(got["n_found"] - len(ro_r)) <= max(2, len(ro_r) // 10)


def test_batch_search_graph_replays_match_eager(dev):
    """A whole pass (several chunks, every job's peaks) recorded once as a HIP
    graph: each replay, on new spectra with eager work and synchronisation in
    between, gives exactly the eager pass's peak lists."""
    import torch
    from paper_2206_12205_amd.pipeline import BatchSearch
    lengths = [20000, 70001, 3001, 150000, 9000, 40000, 1, 131072]
    n_z, M = 9, 128
    say("[pipeline] graph capture of a pass")
    xa = torch.from_numpy(np.concatenate(batch_spectra(lengths, seed=21))).to(dev)
    xb = torch.from_numpy(np.concatenate(batch_spectra(lengths, seed=22))).to(dev)
    bs = BatchSearch(lengths, -8.0, 2.0, n_z, M, compute="bf16", plane_dtype="bf16",
                     buffer_bytes=n_z * 160000 * 2 * 2, tune=False, device=dev, peak_capacity=256)
    assert len(bs.chunks) >= 3
    thr = 20.0

    def lists():
        return [bs.peaks(i) for i in range(len(lengths))]

    want = {}
    for name, src in (("a", xa), ("b", xb)):
        bs.run(src, thr)
        torch.cuda.synchronize()
        want[name] = lists()
    spectra = xa.clone()
    g = bs.capture(spectra, thr)
    for rep, name in enumerate("abab"):
        spectra.copy_(xa if name == "a" else xb)     # eager work between replays
        bs.n_found.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = lists()
        for i, (gi, wi) in enumerate(zip(got, want[name])):
            assert gi["n_found"] == wi["n_found"], f"replay {rep} job {i}"
            for k in ("z_idx", "r", "power"):
                assert np.array_equal(gi[k], wi[k]), f"replay {rep} job {i} {k}"
        _ = float(bs.buffer.float().sum().item())     # more eager work on the same stream
    del g


def test_batch_search_harmonic_sums_match_single_plans(dev):
    """Harmonic sums in the batched search: each job's list for H = 2 and 4
    equals fdas_harmonic_sum_peaks on the plane of a single plan with the
    same knobs (one batched sums call per chunk, the sums never stored)."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    from paper_2206_12205_amd.pipeline import BatchSearch
    lengths = [20000, 70001, 3001, 150000, 1, 40000]
    n_z, M = 9, 128
    say(f"[pipeline] harmonic sums, lengths {lengths}")
    parts = batch_spectra(lengths, seed=21)
    x = torch.from_numpy(np.concatenate(parts)).to(dev)
    harm = {2: 24.0, 4: 30.0}
    bs = BatchSearch(lengths, -8.0, 2.0, n_z, M, compute="bf16", plane_dtype="bf16",
                     buffer_bytes=n_z * 160000 * 2 * 2, device=dev, peak_capacity=256, harmonics=harm)
    bs.run(x, 20.0)
    torch.cuda.synchronize()
    for i, n in enumerate(lengths):
        cls = max(int(math.ceil(math.log2(n))), 0)
        t = bs.tuned[cls]
        cmax = max(v for v in lengths if max(int(math.ceil(math.log2(v))), 0) == cls)
        pl = Plan(cmax, -8.0, 2.0, n_z, M, t["seg_len"], compute="bf16", plane_dtype="bf16", algo=t["algo"],
                  z_chunk=t["z_chunk"], device=dev)
        P = pl.correlate(torch.from_numpy(parts[i]).to(dev))
        for h, thr in harm.items():
            _, ref = pl.harmonic_sum_peaks(P, h, thr, capacity=256)
            got = bs.peaks(i, h)
            assert got["n_found"] == ref["n_found"], f"job {i} H={h}"
            for k in ("z_idx", "r", "power"):
                assert np.array_equal(got[k], ref[k]), f"job {i} H={h} {k}"
    assert any(bs.peaks(i, 2)["n_found"] > 0 for i in range(len(lengths)))
