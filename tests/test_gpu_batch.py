"""GPU checks of the batched entry point (fdas_set_batch / fdas_correlate_batch).

Many spectra of uneven length (dedispersion trials) go through one launch.
Each job's plane must be bit-identical to what fdas_correlate writes for that
spectrum alone (same kernels, same arithmetic), and a few jobs are also held
against the FP64 oracle to the BF16 bar.  The batch is captured in a HIP graph
and replayed several times, with eager work (new spectra, cleared planes)
between replays; every replay is checked against the eager result.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import plane as OP
from oracle import response as R

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# BF16's segment 4096 with 256 taps keeps V = 3840 valid bins per segment
# (FP32's automatic 2048 keeps V = 1792; 3839..3841 straddle its third segment)
LENGTHS = [70001, 1, 3839, 3840, 3841, 12345, 200000, 517]
ZMIN, ZSTEP, NZ, M = -20.0, 2.0, 21, 256


def make_plan(dev, compute="bf16", plane_dtype="bf16", algo="auto", max_jobs=len(LENGTHS), z_chunk=0):
    from paper_2206_12205_amd.fdas import Plan
    return Plan(max_bins=max(LENGTHS), z_min=ZMIN, z_step=ZSTEP, n_z=NZ, n_taps=M, seg_len=0,
                compute=compute, plane_dtype=plane_dtype, algo=algo, max_jobs=max_jobs,
                z_chunk=z_chunk, device=dev)


def packed(lengths, seed):
    import torch
    x = synth.random_spectrum(int(sum(lengths)), seed=seed)
    return x, torch.from_numpy(x.astype(np.complex64)).to("cuda:0")


def single(pl, x_host, so, nb):
    import torch
    xi = torch.from_numpy(np.ascontiguousarray(x_host[so:so + nb], dtype=np.complex64)).to(pl.device)
    return pl.correlate(xi)


@pytest.mark.parametrize("compute,plane_dtype,algo", [
    ("bf16", "bf16", "auto"),     # persistent matrix-core launch
    ("bf16", "fp32", "auto"),
    ("fp32", "fp32", "auto"),     # one vector-ALU launch per job
    ("bf16", "bf16", "valu"),
])
def test_batch_equals_single(dev, compute, plane_dtype, algo):
    import torch
    say(f"[batch] {compute}/{plane_dtype}/{algo} jobs={LENGTHS}")
    pl = make_plan(dev, compute, plane_dtype, algo)
    x, xd = packed(LENGTHS, seed=101)
    offs = pl.set_batch(LENGTHS)
    planes = torch.full((pl.batch_cells,), float("nan"), dtype=pl.torch_plane_dtype(), device=dev)
    pl.correlate_batch(xd, planes)
    torch.cuda.synchronize()
    for i, (nb, (so, po)) in enumerate(zip(LENGTHS, offs)):
        ref = single(pl, x, so, nb)
        got = pl.batch_plane(planes, i)
        assert torch.equal(got, ref), f"job {i} (n={nb}) differs from fdas_correlate"


def test_batch_vs_oracle(dev):
    """Jobs 1, 3841 and 517 bins (the short and ragged ones) against the oracle."""
    import torch
    say("[batch] vs oracle")
    pl = make_plan(dev, "bf16", "fp32")
    x, xd = packed(LENGTHS, seed=102)
    offs = pl.set_batch(LENGTHS)
    planes = pl.correlate_batch(xd)
    torch.cuda.synchronize()
    taps = R.template_taps(R.z_grid(ZMIN, ZSTEP, NZ), M)
    for i in (1, 4, 7):
        nb, (so, _) = LENGTHS[i], offs[i]
        ref = OP.plane(x[so:so + nb], taps)
        got = pl.batch_plane(planes, i).double().cpu().numpy()
        err = np.abs(got - ref) / np.maximum(ref, 1.0)
        assert err.max() <= 0.15 and err.mean() <= 0.02, f"job {i}: max {err.max():.3e}"
        bright = ref > 20.0
        if bright.any():
            assert (np.abs(got[bright] - ref[bright]) / ref[bright]).max() <= 0.03


def test_batch_reset_between_batches(dev):
    """A second, smaller batch on the same plan: the tile counter restarts and
    only the new jobs are written."""
    import torch
    say("[batch] second batch")
    pl = make_plan(dev)
    x, xd = packed(LENGTHS, seed=103)
    pl.set_batch(LENGTHS)
    pl.correlate_batch(xd)
    small = [5000, 7]
    offs = pl.set_batch(small)
    planes = torch.zeros(pl.batch_cells + 1000, dtype=torch.bfloat16, device=dev)
    pl.correlate_batch(xd, planes)
    torch.cuda.synchronize()
    for i, (nb, (so, _)) in enumerate(zip(small, offs)):
        assert torch.equal(pl.batch_plane(planes, i), single(pl, x, so, nb))
    assert torch.count_nonzero(planes[pl.batch_cells:]) == 0


@pytest.mark.parametrize("plane_dtype", ["bf16", "fp32"])
def test_batch_graph_replays(dev, plane_dtype):
    import torch
    say(f"[batch] graph replay {plane_dtype}")
    pl = make_plan(dev, "bf16", plane_dtype)
    lengths = [40000, 3841, 1, 9000]
    pl.set_batch(lengths)
    xa, xda = packed(lengths, seed=104)
    xb, xdb = packed(lengths, seed=105)
    spectra = xda.clone()
    planes = torch.zeros(pl.batch_cells, dtype=pl.torch_plane_dtype(), device=dev)
    # eager results for both inputs
    want_a = pl.correlate_batch(xda).clone()
    want_b = pl.correlate_batch(xdb).clone()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pl.correlate_batch(spectra, planes)           # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pl.correlate_batch(spectra, planes)
    for rep, (src, want) in enumerate([(xda, want_a), (xdb, want_b), (xda, want_a), (xdb, want_b)]):
        spectra.copy_(src)                            # eager work between replays
        planes.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(planes, want), f"replay {rep} differs from the eager batch"
        _ = (planes.float().sum()).item()             # more eager work on the same stream
    del g
