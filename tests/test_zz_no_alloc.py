"""GPU check of fdas_harmonic_sums_peaks_noalloc, the entry point for callers
that cannot allocate device memory: through the C ABI, its sums, peak lists
and counts equal those of fdas_harmonic_sums_peaks (caller scratch) on the
same plane, bit for bit, on two calls in a row, the second with a smaller
plane and fewer sums (the fixed scratch keeps the first call's contents)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def noise_plane(dev, n_z, n, seed, dtype):
    """Exp(1) noise (the normalised plane's distribution) with a few bright
    cells, in the plane dtype."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    P = -torch.log1p(-torch.rand((n_z, n), generator=g, dtype=torch.float64))
    rows = torch.randint(0, n_z, (40,), generator=g)
    cols = torch.randint(0, n, (40,), generator=g)
    P[rows, cols] = 30.0 + 60.0 * torch.rand(40, generator=g, dtype=torch.float64)
    return P.to(dtype).to(dev).contiguous()


def run_pair(pl, P, hs, thr, cap):
    """The same sums and lists through both entry points -> (sums_a, lists_a,
    counts_a, sums_b, lists_b, counts_b)."""
    import torch
    dev = P.device
    n = P.shape[1]
    out = {}
    for which in ("scratch", "noalloc"):
        outs = [torch.full((pl.n_z, (n - 1) // h + 1), float("nan"), dtype=P.dtype, device=dev) for h in hs]
        pk = torch.zeros((len(hs), cap, 24), dtype=torch.uint8, device=dev)
        nf = torch.full((len(hs),), -1, dtype=torch.int64, device=dev)
        peaks = [(pk[l].data_ptr(), cap) for l in range(len(hs))]
        if which == "scratch":
            scr = torch.empty(pl.harmonic_sums_peaks_bytes(n, hs), dtype=torch.uint8, device=dev)
            pl.harmonic_sums_peaks_async(P.data_ptr(), n, hs, thr, [o.data_ptr() for o in outs], peaks,
                                         nf.data_ptr(), scr)
        else:
            pl.harmonic_sums_peaks_noalloc_async(P.data_ptr(), n, hs, thr, [o.data_ptr() for o in outs], peaks,
                                                 nf.data_ptr())
        torch.cuda.synchronize(dev)
        out[which] = (outs, pk.cpu(), nf.cpu().tolist())
    return out["scratch"], out["noalloc"]


@pytest.mark.parametrize("plane_dtype", ["bf16", "fp32"])
def test_noalloc_sums_peaks_equal_scratch_entry(dev, plane_dtype):
    import torch
    from paper_2206_12205_amd import fdas as F
    from paper_2206_12205_amd.fdas import Plan
    tdt = {"bf16": torch.bfloat16, "fp32": torch.float32}[plane_dtype]
    n_z, n1, n2 = 101, 1_000_003, 300_001
    pl = Plan(max_bins=n1, z_min=-100.0, z_step=2.0, n_z=n_z, n_taps=256, compute="bf16", plane_dtype=plane_dtype,
              device=dev)
    cap = 4096
    calls = [(n1, [2, 4, 8, 16], [14.0, 18.0, 26.0, 40.0], 1),
             (n2, [2, 8], [12.0, 22.0], 2)]          # second call: smaller plane, fewer sums
    for n, hs, thr, seed in calls:
        say(f"[noalloc] {plane_dtype} n_z {n_z} n {n} H {hs}")
        need = pl.harmonic_sums_peaks_bytes(n, hs)
        assert need <= F.NOALLOC_SCRATCH_BYTES
        P = noise_plane(dev, n_z, n, seed, tdt)
        (sa, pa, ca), (sb, pb, cb) = run_pair(pl, P, hs, thr, cap)
        assert ca == cb, f"counts {ca} vs {cb}"
        assert all(0 < c <= cap for c in ca), ca
        for l, h in enumerate(hs):
            assert torch.equal(sa[l].view(torch.int16 if tdt == torch.bfloat16 else torch.int32),
                               sb[l].view(torch.int16 if tdt == torch.bfloat16 else torch.int32)), f"sum H={h}"
            k = ca[l]
            assert torch.equal(pa[l, :k], pb[l, :k]), f"list H={h}"
            rec = pb[l, :k].numpy().view(np.dtype([("r", "<i8"), ("z_idx", "<i4"), ("job", "<i4"),
                                                    ("power", "<f4"), ("reserved", "<f4")])).reshape(-1)
            key = rec["z_idx"].astype(np.int64) * (n + 1) + rec["r"]
            assert np.all(np.diff(key) > 0), f"list H={h} not sorted by (z, r)"
