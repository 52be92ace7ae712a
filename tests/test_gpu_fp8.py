"""GPU checks of the FP8 (OCP e4m3) precision form.

Bars.  The bank must hold the oracle's e4m3 values of the FP32-rounded
template spectra scaled by the same power of two (one e4m3 step apart in rare
cases where the GPU's and the oracle's FP64 spectra round to different FP32
values; the sign of an exact zero is not compared).  The plane is held against the FP64 oracle with bars from the
e4m3 rounding: each rounding is at most 2^-4 of the value; along the path
there are six (two forward stages, the segment spectrum, the template, two
inverse stages) with power-of-two scales set from each stage's largest
component, so cells that carry a bright signal see a few per cent and cells
near the noise floor up to about one noise unit: bright cells (P64 > 20)
within 10 %, every cell within 1.0 max(P64, 1), mean within 0.10 max(P64, 1).
The brightest cell of an injected signal must be the oracle's.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import casts
from oracle import plane as OP
from oracle import response as R

pytestmark = pytest.mark.gpu

C1 = synth.CONFIGS[1]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def plan(dev, **kw):
    from paper_2206_12205_amd.fdas import Plan
    return Plan(device=dev, **kw)


def test_fp8_bank_matches_oracle(dev):
    import torch
    say("[fp8] bank")
    zs = R.z_grid(C1["z_min"], C1["z_step"], C1["n_z"])
    for L in (1024, 4096):
        pl = plan(dev, max_bins=65536, z_min=C1["z_min"], z_step=C1["z_step"], n_z=C1["n_z"],
                  n_taps=C1["n_taps"], seg_len=L, compute="fp8")
        torch.cuda.synchronize()
        codes = pl.bank().cpu().numpy()                 # (n_z, L, 2) uint8
        texp = pl.fp8_exponents().cpu().numpy()
        H = R.template_spectra(zs, C1["n_taps"], L)
        h32 = np.stack([H.real, H.imag], axis=-1).astype(np.float32).astype(np.float64)
        hmax = np.abs(h32).reshape(C1["n_z"], -1).max(axis=1)
        t_ref = np.floor(np.log2(448.0 / hmax)).astype(np.int64)
        assert np.array_equal(texp, t_ref)
        want = casts.e4m3_bits(h32 * np.ldexp(1.0, t_ref)[:, None, None])
        # compare values, not codes: +0 and -0 are the same value (the z = 0
        # template's imaginary parts are exact zeros on the GPU and +-1e-17
        # rounding noise in the oracle's FFT)
        got_v, want_v = casts.e4m3_decode(codes), casts.e4m3_decode(want)
        step = np.spacing(np.maximum(np.abs(want_v), 2.0 ** -6).astype(np.float32)) * 2.0 ** 20   # one e4m3 step
        d = np.abs(got_v - want_v)
        assert np.all(d <= step), f"L={L}: {d.max()}"
        assert np.mean(d != 0) < 1e-3, f"L={L}: {np.mean(d != 0)}"


def fp8_plane_vs_oracle(dev, x, zmin, zstep, nz, M, L, pd="fp32"):
    taps = R.template_taps(R.z_grid(zmin, zstep, nz), M)
    ref = OP.plane(x, taps)
    import torch
    pl = plan(dev, max_bins=x.size, z_min=zmin, z_step=zstep, n_z=nz, n_taps=M, seg_len=L, compute="fp8",
              plane_dtype=pd)
    p = pl.correlate(torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to(dev)).double().cpu().numpy()
    return p, ref


def check_fp8(p, ref, what):
    err = np.abs(p - ref) / np.maximum(ref, 1.0)
    assert np.all(np.isfinite(p)), what
    assert err.max() <= 1.0, f"{what}: max {err.max():.3f}"
    assert err.mean() <= 0.10, f"{what}: mean {err.mean():.3f}"
    bright = ref > 20.0
    if bright.any():
        rb = np.abs(p[bright] - ref[bright]) / ref[bright]
        assert rb.max() <= 0.10, f"{what}: bright {rb.max():.3f}"
    return err


@pytest.mark.parametrize("L,pd", [(4096, "fp32"), (2048, "bf16"), (1024, "fp32")])
def test_fp8_plane_tiny_workload(dev, L, pd):
    say(f"[fp8] tiny workload L={L} {pd}")
    sp = synth.config1(0)
    x = sp.spec[:30000]
    p, ref = fp8_plane_vs_oracle(dev, x, C1["z_min"], C1["z_step"], C1["n_z"], C1["n_taps"], L, pd)
    err = check_fp8(p, ref, f"L={L}")
    say(f"  max {err.max():.3f} mean {err.mean():.4f}")
    assert np.unravel_index(np.argmax(p), p.shape) == np.unravel_index(np.argmax(ref), ref.shape)


@pytest.mark.parametrize("n,M", [(1, 64), (3840, 256), (3841, 256), (9001, 130)])
def test_fp8_edge_shapes(dev, n, M):
    say(f"[fp8] n={n} M={M}")
    x = synth.random_spectrum(n, seed=n + M)
    p, ref = fp8_plane_vs_oracle(dev, x, -6.0, 3.0, 5, M, 4096)
    check_fp8(p, ref, f"n={n}")


def test_fp8_chirp_peak(dev):
    say("[fp8] chirp")
    n_t, r_bar, z = 1 << 16, 12345, 20.0
    x = synth.complex_chirp_spectrum(n_t, r_bar - z / 2, z, amp=0.05)
    p, ref = fp8_plane_vs_oracle(dev, x, -40.0, 4.0, 21, 256, 4096)
    assert np.unravel_index(np.argmax(p), p.shape) == np.unravel_index(np.argmax(ref), ref.shape)
    assert abs(p.max() / ref.max() - 1.0) < 0.10


def test_fp8_nan_poisons_its_segments(dev):
    """A NaN bin makes every output of the segments that read it NaN (the
    e4m3 format has no infinities; NaN stays NaN)."""
    import torch
    say("[fp8] NaN")
    n, M, L = 20000, 256, 4096
    V = L - M
    x = synth.random_spectrum(n, seed=5)
    x[9000] = np.nan
    pl = plan(dev, max_bins=n, z_min=-4.0, z_step=4.0, n_z=3, n_taps=M, seg_len=L, compute="fp8")
    p = pl.correlate(torch.from_numpy(x).to(dev)).cpu().numpy()
    bad = np.isnan(p).all(axis=0)
    segs = [s for s in range((n + V - 1) // V) if s * V - M // 2 <= 9000 < s * V - M // 2 + L]
    cols = np.zeros(n, bool)
    for s in segs:
        cols[s * V:min((s + 1) * V, n)] = True
    assert np.array_equal(bad, cols)
