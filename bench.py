#!/usr/bin/env python3
"""Benchmark of the FDAS hot path: f-fdot plane cells/s, BF16 vs FP32, on one GPU.

Workload (single-DM): 2^23 samples at 64 us -> 4,194,304 complex bins,
101 templates (z in [-100, 100] step 2), 256 taps, one injected 8-harmonic
binary pulsar (seeded, synthetic).  A step is one fdas_correlate of the whole
plane (101 x 4,194,304 cells) with the spectrum already resident in device
memory.  The headline value is the BF16 form (bfloat16 storage, FP32
accumulation, raw bfloat16 plane) at the library's segment length (4096);
segment 8192 (the workload's stated length), the vector-ALU BF16 kernel and
the FP32 form are timed beside it.  Accuracy (outside the timed region): band
maxima of a seeded trial ensemble against the FP64 plane.

Prints one JSON line.  --gpus N > 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
T_START = time.perf_counter()


def note(msg):
    """Progress of the run on stderr (the result is the one JSON line on stdout)."""
    print(f"[bench {time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


PREROLL_MS = 40.0


def preroll(fn, min_ms=PREROLL_MS):
    """Run fn (one launch) back to back until at least min_ms of device time
    has passed, whatever the warm-up count: the GPU clock needs a few tens of
    milliseconds of steady load to settle, so the timed window then starts at
    the steady clock.  Outside every timed region."""
    import torch
    st = torch.cuda.current_stream()
    spent = 0.0
    while spent < min_ms:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(16):
            fn()
        e1.record(st)
        e1.synchronize()
        spent += e0.elapsed_time(e1)
    return spent


def time_correlate(pl, x, plane, steps, warmup):
    import torch
    preroll(lambda: pl.correlate(x, plane))
    for _ in range(warmup):
        pl.correlate(x, plane)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        pl.correlate(x, plane)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def launch_stats(pl, x, plane, n=256):
    """Mean, standard deviation and median of n individually timed launches
    (HIP events around each launch on the launch stream), in ms."""
    import statistics
    import torch
    st = torch.cuda.current_stream()
    preroll(lambda: pl.correlate(x, plane))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(st)
        pl.correlate(x, plane)
        b.record(st)
    torch.cuda.synchronize()
    t = [a.elapsed_time(b) for a, b in ev]
    return {"mean": statistics.fmean(t), "std": statistics.pstdev(t), "median": statistics.median(t), "n": n}


def fill_bandwidth(dev, nbytes=4 << 30, reps=10):
    """Achieved HBM bandwidth of a plain device fill (write bytes only over
    time): the ceiling for a path whose traffic is almost all plane writes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    for _ in range(3):
        a.fill_(1.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        a.fill_(1.0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a
    return nbytes / (ms * 1e-3) / 1e9


def copy_bandwidth(dev, nbytes=4 << 30, reps=10):
    """Achieved HBM bandwidth of a plain device-to-device copy (read + write
    bytes over time), the practical ceiling next to the 8 TB/s peak."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def measured_counts(kernel_sources):
    """Per-launch instruction counts from the committed counter summary (same
    source-hash guard as the traffic), or None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "correlate_mfma4096_single_dm_hbm_counters.md")
    try:
        txt = open(path).read()
        h = hashlib.sha1()
        for f in kernel_sources:
            with open(os.path.join(ROOT, "paper_2206_12205_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if re.search(r"kernel_source_sha1: ([0-9a-f]+)", txt).group(1) != h.hexdigest():
            return None
        return {k: float(re.search(rf"{k}: ([0-9.e+]+)", txt).group(1))
                for k in ("mfma_insts_per_launch", "valu_insts_per_launch")}
    except (OSError, AttributeError):
        return None


def measured_traffic(kernel_sources):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources no longer hash to the profiled version."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "correlate_mfma4096_single_dm_hbm_counters.md")
    try:
        txt = open(path).read()
        h = hashlib.sha1()
        for f in kernel_sources:
            with open(os.path.join(ROOT, "paper_2206_12205_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        sha = re.search(r"kernel_source_sha1: ([0-9a-f]+)", txt).group(1)
        if sha != h.hexdigest():
            return None
        return int(re.search(r"traffic_bytes_per_launch: (\d+)", txt).group(1))
    except (OSError, AttributeError):
        return None


def cpu_baseline(spec, cfg, r_center, target_s=15.0):
    """The FP64 oracle (direct correlation, OpenMP over r) on a window of
    columns x all template rows, sized for ~target_s of CPU work."""
    from oracle import plane as oplane
    from oracle import response as oresp
    zs = oresp.z_grid(cfg["z_min"], cfg["z_step"], cfg["n_z"])
    taps = oresp.template_taps(zs, cfg["n_taps"])
    w = 16384
    a = max(r_center - w // 2, 0)
    oplane.plane(spec, taps, a, a + 1024)          # start the OpenMP pool
    t = time.perf_counter()
    oplane.plane(spec, taps, a, a + w)
    dt = time.perf_counter() - t
    w2 = int(min(max(w * target_s / max(dt, 1e-3), w), spec.size))
    a = max(min(r_center - w2 // 2, spec.size - w2), 0)
    t = time.perf_counter()
    oplane.plane(spec, taps, a, a + w2)
    dt = time.perf_counter() - t
    cells = w2 * cfg["n_z"]
    return {"value": cells / dt, "unit": "cells/s", "cores": oplane.threads(), "kind": "oracle",
            "sample": f"FP64 direct correlation, columns [{a}, {a + w2}) x {cfg['n_z']} templates "
                      f"({cells} cells, {dt:.1f} s), {cfg['n_taps']} taps"}


def batched_search(args, cfg, dev):
    """Many-spectra workload: 256 dedispersion trials with series lengths
    log-uniform in [2^20, 2^23] samples, even counts (spectra of 2^19..2^22
    bins, any length in between), 10 % of
    them with an injected binary pulsar, generated on the device (seeded);
    the single-DM template grid, BF16 form, autotuned plan per length class,
    planes chunked through a 16 GB buffer and thresholded peaks of every
    plane."""
    import numpy as np
    import torch
    import synth
    from paper_2206_12205_amd.pipeline import BatchSearch
    c3 = synth.CONFIGS[3]
    note("batched: generating 256 trials on the device")
    spectra, trials = synth.config3(dev)
    lengths = [t.n_bins for t in trials]
    note("batched: trials ready; planning and tuning")
    total = int(sum(lengths))
    t0 = time.perf_counter()
    harm = {2: c3["threshold"] + 10, 4: c3["threshold"] + 20, 8: c3["threshold"] + 30, 16: c3["threshold"] + 40}
    bs = BatchSearch(lengths, c3["z_min"], c3["z_step"], c3["n_z"], c3["n_taps"], compute="bf16",
                     plane_dtype="bf16", buffer_bytes=16 << 30, tune=True, device=dev, harmonics=harm)
    bs.harmonics = {}                      # plane and peaks only, until the harmonic timing below
    setup_s = time.perf_counter() - t0
    note(f"batched: {len(trials)} trials generated, {len(bs.chunks)} chunks planned and tuned ({setup_s:.1f} s)")
    res = {}
    for name, fp, fu in (("correlate", False, True), ("correlate_and_peaks_per_job", True, False),
                         ("correlate_and_peaks", True, True)):
        bs.run(spectra, c3["threshold"], find_peaks=fp, fused=fu)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        steps = max(1, min(args.steps, 3))
        e0.record()
        for _ in range(steps):
            bs.run(spectra, c3["threshold"], find_peaks=fp, fused=fu)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"ms_per_pass": ms, "cells_per_s": bs.cells / (ms * 1e-3)}
        note(f"batched {name}: {ms:.1f} ms per pass")
    # the same pass recorded once as a HIP graph and replayed
    g = bs.capture(spectra, c3["threshold"], find_peaks=True)
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steps = max(1, min(args.steps, 3))
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res["correlate_and_peaks_graph"] = {"ms_per_pass": ms, "cells_per_s": bs.cells / (ms * 1e-3),
                                        "launches_per_pass": len(bs.chunks) * 7}
    note(f"batched correlate_and_peaks as one HIP graph: {ms:.1f} ms per pass")
    del g
    # the full search of every trial: plane with peaks, then the sums over
    # H = 2, 4, 8, 16 harmonics of every plane with their peaks
    bs.harmonics = harm
    bs.run(spectra, c3["threshold"])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        bs.run(spectra, c3["threshold"])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # per chunk: 7 launches of the correlation with its peaks, 5 of the
    # batched harmonic sums with their peaks (layout, sums and marks, count,
    # scan, write)
    res["correlate_peaks_and_harmonic_sums"] = {
        "ms_per_pass": ms, "harmonics": {str(h): t for h, t in harm.items()},
        "harmonic_sums_ms_per_pass": ms - res["correlate_and_peaks"]["ms_per_pass"],
        "launches_per_pass": len(bs.chunks) * (7 + 5),
        "harmonic_peaks_found": sum(int(v) for v in bs.hn_found_all.cpu().tolist())}
    note(f"batched plane + peaks + harmonic sums H = 2..16 with peaks: {ms:.1f} ms per pass")
    bs.harmonics = {}
    # an injected pulsar counts as found when a peak sits within 2 bins of
    # the mean frequency of one of its harmonics
    found, noise_peaks, injected = 0, 0, 0
    for i, t in enumerate(trials):
        pk = bs.peaks(i)
        if t.pulsar is None:
            noise_peaks += pk["n_found"]
            continue
        injected += 1
        rb = [t.pulsar.r_bar(t.T, h) for h in range(1, len(t.pulsar.amps) + 1) if t.pulsar.amps[h - 1] > 0]
        if pk["n_found"] and any(np.min(np.abs(pk["r"] - r)) <= 2 for r in rb):
            found += 1
    out = {"workload": f"{len(trials)} dedispersion trials, series log-uniform in [2^20, 2^23] samples "
                       f"(even counts) "
                       f"(spectra {min(lengths)}..{max(lengths)} bins, total {total}), 10 % with an injected "
                       f"binary pulsar, {c3['n_z']} templates, {c3['n_taps']} taps, BF16 form, raw BF16 "
                       f"planes chunked through a 16 GB buffer, peaks above {c3['threshold']}",
           "cells": bs.cells, "chunks": len(bs.chunks), "setup_s": setup_s,
           "tuned": {f"2^{k}": v for k, v in bs.tuned.items()},
           "injected_pulsars": injected, "pulsars_with_a_harmonic_peak": found,
           "peaks_in_noise_only_trials": noise_peaks, **res}
    del bs, spectra
    return out


def peaks_timing(pl, x, plane, thr, steps, ms_plane):
    """Plane plus thresholded peaks of the headline spectrum: fdas_correlate
    then fdas_peaks (a streaming pass over the plane flags the tiles) against
    fdas_correlate_peaks (the correlation kernel flags them while storing the
    plane); the same list either way."""
    import ctypes
    import torch
    from paper_2206_12205_amd import fdas as F
    L = F.lib()
    n = x.numel()
    cap = 1 << 16
    out = torch.empty((cap, 24), dtype=torch.uint8, device=x.device)
    nf = torch.zeros(1, dtype=torch.int64, device=x.device)
    xs, pp = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(plane.data_ptr())
    op, np_ = ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(nf.data_ptr())
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)

    def separate():
        F._check(L.fdas_correlate(pl._h, xs, n, pp, sp), "fdas_correlate")
        F._check(L.fdas_peaks(pl._h, pp, n, float(thr), op, cap, np_, sp), "fdas_peaks")

    def fused():
        F._check(L.fdas_correlate_peaks(pl._h, xs, n, pp, float(thr), op, cap, np_, sp), "fdas_correlate_peaks")

    res = {}
    for name, fn in (("correlate_then_peaks", separate), ("correlate_peaks_fused", fused)):
        preroll(fn)
        for _ in range(max(steps // 4, 5)):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # ms_over_plane: this timing minus the plane-only timing of the same
        # plan (two measurements: box noise of a few us either way)
        res[name] = {"ms": ms, "cells_per_s": pl.n_z * n / (ms * 1e-3), "ms_over_plane": ms - ms_plane,
                     "n_found": int(nf.item())}
    res["threshold"] = thr
    note(f"plane + peaks: separate {res['correlate_then_peaks']['ms']:.4f} ms, "
         f"fused {res['correlate_peaks_fused']['ms']:.4f} ms ({res['correlate_peaks_fused']['n_found']} peaks)")
    return res


def harmonic_timing(pl, plane, steps, thr):
    """fdas_harmonic_sum on the headline BF16 plane for H = 2, 4, 8, 16:
    time per call, summed cells per second and HBM fraction of the
    algorithmic bytes (the plane read once plus the summed plane written);
    then the sum with thresholded peaks, as fdas_harmonic_sum followed by
    fdas_peaks and as one fdas_harmonic_sum_peaks call."""
    import ctypes
    import torch
    from paper_2206_12205_amd import fdas as F
    L = F.lib()
    n_z, n = plane.shape
    cap = 1 << 16
    pk = torch.empty((cap, 24), dtype=torch.uint8, device=plane.device)
    nf = torch.zeros(1, dtype=torch.int64, device=plane.device)
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    pp, kp, fp = ctypes.c_void_p(plane.data_ptr()), ctypes.c_void_p(pk.data_ptr()), ctypes.c_void_p(nf.data_ptr())

    def timed(fn, reps):
        preroll(fn)
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    elem = plane.element_size()
    res = {}
    for H in (2, 4, 8, 16):
        out = pl.harmonic_sum(plane, H)
        preroll(lambda: pl.harmonic_sum(plane, H, out))
        for _ in range(10):
            pl.harmonic_sum(plane, H, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(10, min(steps, 100))
        e0.record()
        for _ in range(reps):
            pl.harmonic_sum(plane, H, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nh = (n - 1) // H + 1
        alg = n_z * n * elem + n_z * nh * elem
        res[f"H{H}"] = {"ms": ms, "summed_cells_per_s": n_z * nh / (ms * 1e-3),
                        "algorithmic_GBs": alg / (ms * 1e-3) / 1e9,
                        "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        op = ctypes.c_void_p(out.data_ptr())

        def separate():
            F._check(L.fdas_harmonic_sum(pl._h, pp, n, H, op, sp), "fdas_harmonic_sum")
            F._check(L.fdas_peaks(pl._h, op, nh, float(thr), kp, cap, fp, sp), "fdas_peaks")

        def fused():
            F._check(L.fdas_harmonic_sum_peaks(pl._h, pp, n, H, op, float(thr), kp, cap, fp, sp),
                     "fdas_harmonic_sum_peaks")
        res[f"H{H}"]["with_peaks"] = {"threshold": thr, "separate_ms": timed(separate, reps),
                                      "fused_ms": timed(fused, reps), "n_found": int(nf.item())}
        note(f"harmonic sum H={H}: {ms:.3f} ms; with peaks: separate "
             f"{res[f'H{H}']['with_peaks']['separate_ms']:.3f} ms, fused {res[f'H{H}']['with_peaks']['fused_ms']:.3f} ms")
        del out
    # the four sums in one pass (fdas_harmonic_sums) against four calls
    hs = (2, 4, 8, 16)
    outs = pl.harmonic_sums(plane, hs)
    ms1 = timed(lambda: pl.harmonic_sums(plane, hs, outs), max(10, min(steps, 100)))
    res["H2_4_8_16_one_pass"] = {"ms": ms1, "separate_calls_ms": sum(res[f"H{h}"]["ms"] for h in hs)}
    note(f"harmonic sums H = 2, 4, 8, 16 in one pass: {ms1:.3f} ms "
         f"(four calls: {res['H2_4_8_16_one_pass']['separate_calls_ms']:.3f} ms)")
    del outs
    return res


def prep_timing(args, cfg, dev):
    """fdas_prepare on seeded noise series on the device (FP32 samples): the
    single-DM length 2^23 and a 3 * 2^k length of the batched workload.  The
    workspace is allocated once, outside the timed launches.  Algorithmic
    bytes: the series read once and the spectrum written once."""
    import ctypes
    import torch
    from paper_2206_12205_amd import fdas as F
    L = F.lib()
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    reps = max(10, min(args.steps, 100))
    res = {}
    for n_t in (cfg["n_t"], 3 << 21):
        g = torch.Generator(device=dev).manual_seed(12205)
        xs = torch.randn(n_t, dtype=torch.float32, device=dev, generator=g)
        out = torch.empty(n_t // 2, dtype=torch.complex64, device=dev)
        nb = ctypes.c_size_t(0)
        F._check(L.fdas_prepare_workspace(n_t, ctypes.byref(nb)), "fdas_prepare_workspace")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        args_c = (ctypes.c_void_p(xs.data_ptr()), n_t, ctypes.c_void_p(out.data_ptr()),
                  ctypes.c_void_p(ws.data_ptr()), nb.value, sp)

        def one():
            F._check(L.fdas_prepare(*args_c), "fdas_prepare")
        preroll(one)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            one()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg = n_t * 4 + (n_t // 2) * 8
        res[str(n_t)] = {"workload": f"{n_t} FP32 samples -> {n_t // 2} normalised bins", "ms": ms,
                         "algorithmic_GBs": alg / (ms * 1e-3) / 1e9,
                         "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        note(f"spectrum preparation ({n_t} samples): {ms:.4f} ms, "
             f"{res[str(n_t)]['algorithmic_GBs']:.0f} GB/s algorithmic")
        del xs, out, ws
    return res


def series_search_timing(args, cfg, dev, pl):
    """The whole search of one single-DM time series (2^23 FP32 samples of
    the workload's first trial) as one timed unit: fdas_prepare, then
    fdas_correlate_peaks, then the thresholded peaks of the sums over H = 2,
    4, 8, 16 harmonics from one summing pass, the sums not stored
    (fdas_harmonic_peaks; threshold: the workload's for the plane, +10 per
    doubling of H); every buffer allocated beforehand, HIP events around the
    three calls.  The same search with the sums stored
    (fdas_harmonic_sums_peaks) is timed beside it."""
    import ctypes
    import numpy as np
    import torch
    import synth
    from paper_2206_12205_amd import fdas as F
    L = F.lib()
    x, _ = synth.config2_series(0)
    xs = torch.from_numpy(x.astype(np.float32)).to(dev)
    n_t = xs.numel()
    n = n_t // 2
    nb = ctypes.c_size_t(0)
    F._check(L.fdas_prepare_workspace(n_t, ctypes.byref(nb)), "fdas_prepare_workspace")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    spec = torch.empty(n, dtype=torch.complex64, device=dev)
    plane = pl.empty_plane(n)
    hs = (2, 4, 8, 16)
    sums = {h: torch.empty((pl.n_z, (n - 1) // h + 1), dtype=plane.dtype, device=dev) for h in hs}   # stored form
    cap = 1 << 16
    pk = torch.empty((len(hs) + 1, cap, 24), dtype=torch.uint8, device=dev)
    nf = torch.zeros(len(hs) + 1, dtype=torch.int64, device=dev)
    thr = {1: cfg["threshold"], 2: cfg["threshold"] + 10, 4: cfg["threshold"] + 20, 8: cfg["threshold"] + 30,
           16: cfg["threshold"] + 40}
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    V = ctypes.c_void_p

    harr = (ctypes.c_int32 * len(hs))(*hs)
    parr = (ctypes.c_void_p * len(hs))(*[sums[h].data_ptr() for h in hs])
    tarr = (ctypes.c_float * len(hs))(*[float(thr[h]) for h in hs])
    karr = (ctypes.c_void_p * len(hs))(*[pk[i].data_ptr() for i in range(1, len(hs) + 1)])
    scr = torch.empty(max(pl.harmonic_sums_peaks_bytes(n, hs), pl.harmonic_peaks_bytes(n, hs), 1),
                      dtype=torch.uint8, device=dev)

    def one(stored=False):
        F._check(L.fdas_prepare(V(xs.data_ptr()), n_t, V(spec.data_ptr()), V(ws.data_ptr()), nb.value, sp),
                 "fdas_prepare")
        F._check(L.fdas_correlate_peaks(pl._h, V(spec.data_ptr()), n, V(plane.data_ptr()), float(thr[1]),
                                        V(pk[0].data_ptr()), cap, V(nf[0:1].data_ptr()), sp), "fdas_correlate_peaks")
        if stored:
            F._check(L.fdas_harmonic_sums_peaks(pl._h, V(plane.data_ptr()), n, len(hs), harr, parr, tarr, karr,
                                                cap, V(nf[1:].data_ptr()), V(scr.data_ptr()), scr.numel(), sp),
                     "fdas_harmonic_sums_peaks")
        else:
            F._check(L.fdas_harmonic_peaks(pl._h, V(plane.data_ptr()), n, len(hs), harr, tarr, V(pk[1].data_ptr()),
                                           cap, V(nf[1:].data_ptr()), V(scr.data_ptr()), scr.numel(), sp),
                     "fdas_harmonic_peaks")

    def timed(stored):
        for _ in range(5):
            one(stored)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(10, min(args.steps, 50))
        e0.record(st)
        for _ in range(reps):
            one(stored)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_stored = timed(True)
    found_stored = nf.cpu().tolist()
    ms = timed(False)
    found = nf.cpu().tolist()
    note(f"whole series search (prepare, plane + peaks, H = 2..16 sums' peaks): {ms:.3f} ms "
         f"({ms_stored:.3f} ms with the sums stored)")
    return {"workload": f"{n_t} FP32 samples -> normalised spectrum -> {pl.n_z} x {n} BF16 plane with peaks -> "
                        f"peaks of the harmonic sums H = 2, 4, 8, 16 (sums not stored)", "ms": ms,
            "ms_sums_stored": ms_stored, "same_counts_as_stored": found == found_stored,
            "thresholds": {str(k): v for k, v in thr.items()},
            "n_found": {"H1": found[0], **{f"H{h}": found[i] for i, h in enumerate(hs, 1)}}}


def refinement_timing(cfg, dev, x, steps):
    """Candidate refinement of the single-DM spectrum: the 4,096 highest
    local maxima of its FP32 plane, each moved by a seeded offset
    (U[-0.5, 0.5] in r, U[-1, 1] in z), 20 ascent steps of the 32-tap
    interpolated power with its analytic gradient (fdas_refine), and the
    backward kernel alone (fdas_refine_backward on the same points).  Device
    buffers are allocated once; the start points are restored outside the
    timed launches."""
    import ctypes
    import numpy as np
    import torch
    import synth
    from paper_2206_12205_amd import fdas as F
    from paper_2206_12205_amd.fdas import Plan
    L = F.lib()
    n = x.numel()
    pl = Plan(max_bins=n, z_min=cfg["z_min"], z_step=cfg["z_step"], n_z=cfg["n_z"], n_taps=cfg["n_taps"],
              seg_len=0, compute="fp32", plane_dtype="fp32", device=dev)
    pk = pl.peaks(pl.correlate(x), 8.0, capacity=1 << 20)
    n_cand, n_steps, taps = 4096, 20, 32
    top = np.argsort(-pk["power"], kind="stable")[:n_cand]
    dr, dz = synth.refine_offsets(n_cand)
    r0 = torch.from_numpy(pk["r"][top].astype(np.float64) + dr).to(dev)
    z0 = torch.from_numpy(cfg["z_min"] + cfg["z_step"] * pk["z_idx"][top].astype(np.float64) + dz).to(dev)
    del pl
    r, z = r0.clone(), z0.clone()
    P, gr, gz = (torch.empty_like(r0) for _ in range(3))
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    V = lambda t: ctypes.c_void_p(t.data_ptr())

    def ascend():
        F._check(L.fdas_refine(V(x), n, n_cand, V(r), V(z), V(P), V(gr), V(gz), taps, n_steps, 1.0, 1.0, sp),
                 "fdas_refine")

    def backward():
        F._check(L.fdas_refine_backward(V(x), n, n_cand, V(r0), V(z0), V(P), V(gr), V(gz), taps, sp),
                 "fdas_refine_backward")

    def timed(fn, reset):
        total = 0.0
        for i in range(steps + 3):
            if reset:
                r.copy_(r0)
                z.copy_(z0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            e1.synchronize()
            if i >= 3:
                total += e0.elapsed_time(e1)
        return total / steps
    ms_a = timed(ascend, True)
    P_end = P.clone()
    F._check(L.fdas_refine(V(x), n, n_cand, V(r0), V(z0), V(P), V(gr), V(gz), taps, 0, 1.0, 1.0, sp),
             "fdas_refine")
    gain = float((P_end / P).median().item())
    ms_b = timed(backward, False)
    res = {"workload": f"{n_cand} single-DM candidates (highest FP32 plane maxima, seeded offsets), "
                       f"{n_steps} ascent steps, {taps} taps, FP64 positions",
           "ms_20_steps": ms_a, "candidates_per_s": n_cand / (ms_a * 1e-3),
           "candidate_steps_per_s": n_cand * n_steps / (ms_a * 1e-3),
           "backward_ms": ms_b, "median_power_gain": gain}
    note(f"refinement: {n_cand} candidates x {n_steps} steps in {ms_a:.3f} ms "
         f"({res['candidates_per_s']:.3g} candidates/s); backward alone {ms_b:.4f} ms")
    return res


def jerk_volume(args, cfg, dev, x, plane):
    """Jerk search on the single-DM spectrum: five planes w = -60, -30, 0, 30,
    60 (BF16 form, matrix-core kernel), one plan (and template bank) per w,
    built once; the volume time is the five correlations.  The bank build per
    w (quadrature of the cubic-phase response in FP64) is timed apart."""
    import torch
    from paper_2206_12205_amd.fdas import Plan
    ws = (-60.0, -30.0, 0.0, 30.0, 60.0)
    n = x.numel()
    common = dict(max_bins=n, z_min=cfg["z_min"], z_step=cfg["z_step"], n_z=cfg["n_z"], n_taps=cfg["n_taps"],
                  compute="bf16", plane_dtype="bf16", device=dev)
    plans = []
    for w in ws:
        pl = Plan(**common)
        pl.make_templates(w=w)
        plans.append(pl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        plans[-1].make_templates(w=ws[-1])
    e1.record()
    torch.cuda.synchronize()
    ms_bank = e0.elapsed_time(e1) / 3
    for _ in range(20):
        for pl in plans:
            pl.correlate(x, plane)
    torch.cuda.synchronize()
    reps = max(5, min(args.steps, 50))
    e0.record()
    for _ in range(reps):
        for pl in plans:
            pl.correlate(x, plane)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    cells = len(ws) * cfg["n_z"] * n
    note(f"jerk volume: {len(ws)} w planes in {ms:.3f} ms; bank build {ms_bank:.2f} ms per w")
    del plans
    return {"workload": f"single-DM spectrum, w in {list(ws)} x {cfg['n_z']} z x {n} r, BF16 form, one plan "
                        f"per w", "cells": cells, "ms_per_volume": ms, "cells_per_s": cells / (ms * 1e-3),
            "bank_build_ms_per_w": ms_bank}


def noise_canopy(args, cfg, dev):
    """The paper's noise-canopy experiment on synthetic noise-only planes:
    eight single-DM noise spectra (no pulsar), their FP32 and BF16 planes,
    and 48 bands per plane of width 1.5 f T bins (f drawn as the pulsar
    population's fundamental, P ~ U[1, 10] ms) at seeded positions, all rows;
    the highest cell of each band by fdas_band_max.  Reported: the canopy
    (the range of the band maxima per width class), and how often BF16 and
    FP32 pick different cells for the same band (a flip) and by how far."""
    import numpy as np
    import torch
    import synth
    from paper_2206_12205_amd.fdas import Plan
    n_t, tsamp = cfg["n_t"], cfg["tsamp"]
    T = n_t * tsamp
    n = n_t // 2
    common = dict(max_bins=n, z_min=cfg["z_min"], z_step=cfg["z_step"], n_z=cfg["n_z"], n_taps=cfg["n_taps"],
                  device=dev)
    pl_f = Plan(compute="fp32", plane_dtype="fp32", **common)
    pl_b = Plan(compute="bf16", plane_dtype="bf16", **common)
    pf, pb = pl_f.empty_plane(n), pl_b.empty_plane(n)
    g = np.random.default_rng(np.random.SeedSequence([12205, 6]))
    maxima = {"narrow": [], "wide": []}
    flips = drift_r = drift_z = extreme = n_bands = 0
    ms_band = 0.0
    for trial in range(8):
        x = synth._device_spectrum(n_t, tsamp, [], 7000 + trial, dev)
        pl_f.correlate(x, pf)
        pl_b.correlate(x, pb)
        periods = g.uniform(1e-3, 10e-3, size=48)
        widths = np.floor(1.5 * T / periods).astype(np.int64)
        starts = np.array([g.integers(0, n - w) for w in widths], dtype=np.int64)
        windows = [(0, cfg["n_z"], int(s0), int(s0 + w)) for s0, w in zip(starts, widths)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bf = pl_f.band_max(pf, windows)
        ms_band += (time.perf_counter() - t0) * 1e3
        bb = pl_b.band_max(pb, windows)
        for k, w in enumerate(widths):
            maxima["narrow" if w < np.median(widths) else "wide"].append(float(bf["power"][k]))
            dz, dr = abs(int(bb["z_idx"][k]) - int(bf["z_idx"][k])), abs(int(bb["r"][k]) - int(bf["r"][k]))
            if dz or dr:
                flips += 1
                drift_r = max(drift_r, dr)
                drift_z = max(drift_z, dz)
                extreme += dz > 1 or dr > 1
        n_bands += len(widths)
    del pl_f, pl_b, pf, pb
    note(f"noise canopy: {n_bands} bands, {flips} BF16/FP32 flips ({extreme} extreme)")
    return {"workload": f"8 single-DM noise-only spectra, FP32 and BF16 planes, {n_bands} bands of width "
                        f"1.5 f T (P ~ U[1, 10] ms), all {cfg['n_z']} rows",
            "canopy_fp32": {k: {"min": min(v), "median": float(np.median(v)), "max": max(v), "bands": len(v)}
                            for k, v in maxima.items()},
            "bf16_vs_fp32_flips": flips, "flips_extreme": extreme, "max_drift_r": drift_r, "max_drift_z": drift_z,
            "bands": n_bands, "band_max_ms_per_plane_host_timed": ms_band / 8}


def wide_search(args, dev):
    """Wide workload: 2^24 samples, 16 injected pulsars, 201 templates (z in
    [-200, 200]), 512 taps; the FP32, BF16 and FP8 planes timed and graded on
    windows around each pulsar's harmonics (r_h +- 32, z_h +- 4) against the
    FP64 plane.  The spectrum is generated on the device (seeded)."""
    import torch
    import synth
    from paper_2206_12205_amd import metrics
    from paper_2206_12205_amd.fdas import Plan
    c5 = synth.CONFIGS[5]
    note("wide: generating the spectrum")
    x, sp = synth.config5_device(dev)
    n = x.numel()
    cells = c5["n_z"] * n
    common = dict(max_bins=n, z_min=c5["z_min"], z_step=c5["z_step"], n_z=c5["n_z"], n_taps=c5["n_taps"],
                  seg_len=0, device=dev)
    forms = {"bf16": Plan(compute="bf16", plane_dtype="bf16", **common),
             "fp32": Plan(compute="fp32", plane_dtype="fp32", **common),
             "fp8": Plan(compute="fp8", plane_dtype="bf16", **common)}
    steps = max(1, min(args.steps, 10))
    out = {"workload": f"wide: {n} bins x {c5['n_z']} templates (z -200..200 step 2), {c5['n_taps']} taps, "
                       f"16 injected pulsars", "cells": cells}
    planes = {}
    for name, pl in forms.items():
        planes[name] = pl.empty_plane(n)
        ms, _ = time_correlate(pl, x, planes[name], steps, 2)
        out[name] = {"value": cells / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms, "seg_len": pl.seg_len,
                     "algo": pl.algo}
        note(f"wide {name}: {ms:.3f} ms per plane")
    pd = Plan(compute="fp64", plane_dtype="fp64", **common).correlate(x)
    note("wide: FP64 plane done")
    std = {k: float(v.to(torch.float32).std()) for k, v in planes.items()}
    acc = {k: {"same_bin": 0, "dsnr": []} for k in planes}
    n_bright = 0
    for psr in sp.pulsars:
        # windows around each harmonic (Table 3 bands of 16 pulsars overlap)
        wins = metrics.pulsar_windows(psr, sp.T, n, c5["z_min"], c5["z_step"], c5["n_z"])
        md = metrics.window_maxima(pd, wins)
        mx = {k: metrics.window_maxima(v.to(torch.float32), wins) for k, v in planes.items()}
        br = [i for i, m in enumerate(mx["fp32"]) if m[2] > c5["threshold"]]
        n_bright += len(br)
        for k in planes:
            acc[k]["same_bin"] += sum((mx[k][i][0], mx[k][i][1]) == (md[i][0], md[i][1]) for i in br)
            acc[k]["dsnr"] += [float(metrics.rel_diff_pct(mx[k][i][2] / std[k], mx["fp32"][i][2] / std["fp32"]))
                               for i in br]
    out["bright_harmonic_windows"] = n_bright
    for k in planes:
        err = ((planes[k].to(torch.float64) - pd).abs() / pd.clamp(min=1.0)).max().item()
        out[k].update({"same_bin_vs_fp64": acc[k]["same_bin"],
                       "max_abs_dsnr_pct_vs_fp32": max(map(abs, acc[k]["dsnr"])) if acc[k]["dsnr"] else None,
                       "max_rel_power_err_vs_fp64": err})
    del pd, planes, forms, x
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed launches before each timed window (after a pre-roll of at least "
                         f"{PREROLL_MS:.0f} ms of device time that brings the GPU clock to its steady state)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched many-spectra search (256 dedispersion trials)")
    ap.add_argument("--no-harmonic", action="store_true", help="skip the harmonic-sum timing")
    ap.add_argument("--no-jerk", action="store_true", help="skip the jerk-volume timing")
    ap.add_argument("--no-refine", action="store_true", help="skip the candidate-refinement timing")
    ap.add_argument("--no-canopy", action="store_true", help="skip the noise-canopy experiment")
    ap.add_argument("--no-prep", action="store_true", help="skip the spectrum-preparation timing")
    ap.add_argument("--no-series", action="store_true", help="skip the whole-series search timing")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the wide workload (201 x 8.4M planes in FP32, BF16 and FP8 vs FP64)")
    ap.add_argument("--trials", type=int, default=256,
                    help="seeded single-DM trials in the accuracy ensemble (outside the timed region)")
    ap.add_argument("--seg-len", type=int, default=None,
                    help="segment length of the BF16 matrix-core plan (default: the workload's 8192)")
    ap.add_argument("--z-chunk", type=int, default=0,
                    help="templates per workgroup of the BF16 plan (0: the library's choice)")
    ap.add_argument("--only", choices=["bf16", "bf16_valu", "fp32", "copy"], default=None,
                    help="time one kernel only (for profiler runs); 'copy' is a plain 256 MiB "
                         "device copy used to calibrate the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this FDAS build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.only == "copy":
        import torch
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"only": "copy", "bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4}))
        return

    import numpy as np
    import torch

    import synth
    from paper_2206_12205_amd import metrics
    from paper_2206_12205_amd.fdas import Plan

    cfg = synth.CONFIGS[2]
    dev = torch.device("cuda:0")
    sp = synth.config2(0)
    n = sp.spec.size
    n_z = cfg["n_z"]
    x = torch.from_numpy(sp.spec).to(dev)
    cells = n_z * n

    common = dict(max_bins=n, z_min=cfg["z_min"], z_step=cfg["z_step"], n_z=n_z,
                  n_taps=cfg["n_taps"], seg_len=cfg["seg_len"], device=dev)
    if args.only:
        kw = {"bf16": dict(compute="bf16", plane_dtype="bf16", seg_len=args.seg_len or cfg["seg_len"],
                           z_chunk=args.z_chunk),
              "bf16_valu": dict(compute="bf16", plane_dtype="bf16", algo="valu"),
              "fp32": dict(compute="fp32", plane_dtype="fp32")}[args.only]
        cm = dict(common)
        cm.update(kw)
        pl = Plan(**cm)
        ms, wall = time_correlate(pl, x, pl.empty_plane(n), args.steps, args.warmup)
        print(json.dumps({"only": args.only, "algo": pl.algo, "seg_len": pl.seg_len,
                          "z_chunk": int(pl.layout.z_chunk), "ms_per_step": ms,
                          "cells_per_s": cells / (ms * 1e-3), "steps": args.steps}), flush=True)
        return
    cm_auto = dict(common)
    cm_auto["seg_len"] = 0                                                 # the library's choice
    pl_b = Plan(compute="bf16", plane_dtype="bf16", **cm_auto)             # matrix-core kernel
    pl_8 = Plan(compute="bf16", plane_dtype="bf16", algo="mfma", **common)  # the stated segment 8192
    pl_v = Plan(compute="bf16", plane_dtype="bf16", algo="valu", **common)
    cm_f = dict(common)
    cm_f["seg_len"] = 0                                                    # the library's choice
    pl_f = Plan(compute="fp32", plane_dtype="fp32", **cm_f)
    pl_q = Plan(compute="fp8", plane_dtype="bf16", **cm_auto)               # FP8 e4m3 form
    plane_b = pl_b.empty_plane(n)
    plane_f = pl_f.empty_plane(n)
    torch.cuda.synchronize()

    note("single-DM spectrum ready; timing the BF16 matrix-core plane")
    ms_b, wall_b = time_correlate(pl_b, x, plane_b, args.steps, args.warmup)
    ms_8, _ = time_correlate(pl_8, x, pl_8.empty_plane(n), args.steps, args.warmup)
    ms_v, _ = time_correlate(pl_v, x, pl_v.empty_plane(n), args.steps, args.warmup)
    ms_f, wall_f = time_correlate(pl_f, x, plane_f, args.steps, args.warmup)
    plane_q = pl_q.empty_plane(n)
    ms_q, _ = time_correlate(pl_q, x, plane_q, args.steps, args.warmup)
    note(f"timed: bf16 {ms_b:.3f} ms, bf16 L=8192 {ms_8:.3f} ms, bf16 valu {ms_v:.3f} ms, fp32 {ms_f:.3f} ms, "
         f"fp8 {ms_q:.3f} ms")
    del pl_v, pl_8

    fused_pk = peaks_timing(pl_b, x, plane_b, cfg["threshold"], args.steps, ms_b)
    if not args.no_harmonic:
        harm = harmonic_timing(pl_b, plane_b, args.steps, cfg["threshold"])
    st_b = launch_stats(pl_b, x, plane_b)
    copy_gbs = copy_bandwidth(dev)
    fill_gbs = fill_bandwidth(dev)
    note(f"per-launch BF16 {st_b['mean']:.4f} +- {st_b['std']:.4f} ms (median {st_b['median']:.4f}); "
         f"device copy {copy_gbs:.0f} GB/s, fill {fill_gbs:.0f} GB/s")
    # algorithmic HBM bytes per launch: the plane store plus one read of the
    # complex64 spectrum (templates are served from cache)
    bytes_b = cells * 2 + n * 8
    bytes_f = cells * 4 + n * 8
    ach_b = bytes_b / (ms_b * 1e-3) / 1e9

    out = {
        "metric": "f-fdot plane cells/s, BF16 vs FP32 on 1 MI355X, at peak-bin match vs FP64",
        "value": cells / (ms_b * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_b,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"single-DM FDAS plane: 4,194,304 bins x 101 templates "
                               f"(z -100..100 step 2), 256 taps, BF16 storage / FP32 accumulation, "
                               f"raw BF16 plane; segment {pl_b.seg_len} (the plane does not depend "
                               f"on the segment length; segment 8192 reported as bf16_seg8192)",
                   "n_bins": n, "n_z": n_z, "n_taps": cfg["n_taps"], "seg_len": pl_b.seg_len,
                   "z_chunk": int(pl_b.layout.z_chunk)},
        "roofline": {"bound": "hbm", "achieved": ach_b, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach_b / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(["correlate_m4k.hip", "mfma4096.hpp"])
                                 if pl_b.algo == "mfma" and pl_b.seg_len == 4096 else None),
                     "kernel": f"correlate_{pl_b.algo}{pl_b.seg_len} (BF16 form, raw BF16 plane)",
                     "bytes_per_launch": bytes_b, "copy_frac": ach_b / copy_gbs, "fill_frac": ach_b / fill_gbs},
        "fp32": {"value": cells / (ms_f * 1e-3), "unit": "cells/s", "ms_per_step": ms_f, "seg_len": pl_f.seg_len,
                 "hbm_frac": bytes_f / (ms_f * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "bf16_seg8192": {"value": cells / (ms_8 * 1e-3), "unit": "cells/s", "ms_per_step": ms_8},
        "bf16_valu": {"value": cells / (ms_v * 1e-3), "unit": "cells/s", "ms_per_step": ms_v},
        "fp8": {"value": cells / (ms_q * 1e-3), "unit": "cells/s", "ms_per_step": ms_q,
                "kernel": f"correlate_valu_fp8 (e4m3 stages, segment {pl_q.seg_len}, raw BF16 plane)"},
        "per_launch_ms": st_b,
        "copy_gbs": copy_gbs,
        "fill_gbs": fill_gbs,
        "speedup_bf16_over_fp32": ms_f / ms_b,
        "wall_s": {"bf16": wall_b, "fp32": wall_f},
    }

    cnt = measured_counts(["correlate_m4k.hip", "mfma4096.hpp"]) if pl_b.algo == "mfma" and pl_b.seg_len == 4096 \
        else None
    if cnt:
        # MFMA: 16x16x32 bf16 = 16,384 flops per instruction against the dense
        # bf16 peak; VALU: wave64 instructions at 4 cycles on a 16-lane SIMD
        # against 1,024 SIMDs at the 2.4 GHz peak clock
        out["utilisation"] = {
            "mfma_frac_of_bf16_peak": cnt["mfma_insts_per_launch"] * 16384 / (ms_b * 1e-3) / 2.5e15,
            "valu_issue_frac_at_peak_clock": cnt["valu_insts_per_launch"] * 4 / (ms_b * 1e-3) / (1024 * 2.4e9),
            "source": "instruction counts of profiles/correlate_mfma4096_single_dm_hbm_counters.md"}

    if not args.no_accuracy:
        # peak-bin match of BF16 and FP32 against the FP64 gold plane on the
        # harmonic bands (Table 3) of each trial's injected pulsar, over a
        # seeded ensemble; SNR differences by Eq. 2 (SNR = power / plane std)
        pl_d = Plan(compute="fp64", plane_dtype="fp64", **common)
        n_bright = same_b = same_f = same_q = 0
        dsnr, dsnr_q, err_b, err_f, err_q = [], [], 0.0, 0.0, 0.0
        for trial in range(args.trials):
            xt, spt = synth.config2_device(dev, trial)
            pd = pl_d.correlate(xt)
            pb = pl_b.correlate(xt, plane_b).to(torch.float32)
            pf = pl_f.correlate(xt, plane_f)
            pq = pl_q.correlate(xt, plane_q).to(torch.float32)
            psr = spt.pulsars[0]
            bands = metrics.harmonic_bands(psr.f, spt.T, n, 8)
            md = metrics.band_maxima(pd, bands)
            mb = metrics.band_maxima(pb, bands)
            mf = metrics.band_maxima(pf, bands)
            mq = metrics.band_maxima(pq, bands)
            sb, sf, sq = float(pb.std()), float(pf.std()), float(pq.std())
            bright = [i for i, m in enumerate(mf) if m[2] > cfg["threshold"]]
            n_bright += len(bright)
            same_b += sum((mb[i][0], mb[i][1]) == (md[i][0], md[i][1]) for i in bright)
            same_f += sum((mf[i][0], mf[i][1]) == (md[i][0], md[i][1]) for i in bright)
            same_q += sum((mq[i][0], mq[i][1]) == (md[i][0], md[i][1]) for i in bright)
            dsnr += [float(metrics.rel_diff_pct(mb[i][2] / sb, mf[i][2] / sf)) for i in bright]
            dsnr_q += [float(metrics.rel_diff_pct(mq[i][2] / sq, mf[i][2] / sf)) for i in bright]
            # max relative power error vs FP64 (floor 1: the noise mean)
            err_b = max(err_b, ((pb.to(torch.float64) - pd).abs() / pd.clamp(min=1.0)).max().item())
            err_f = max(err_f, ((pf.to(torch.float64) - pd).abs() / pd.clamp(min=1.0)).max().item())
            err_q = max(err_q, ((pq.to(torch.float64) - pd).abs() / pd.clamp(min=1.0)).max().item())
            del pd, pb, pq, xt
            if trial % 32 == 31 or trial == args.trials - 1:
                note(f"accuracy trial {trial}: {n_bright} bright band maxima so far")
        out["accuracy"] = {"trials": args.trials, "bright_band_maxima": n_bright,
                           "bf16_same_bin_vs_fp64": same_b, "fp32_same_bin_vs_fp64": same_f,
                           "bf16_same_bin_frac": same_b / n_bright if n_bright else None,
                           "bf16_max_abs_dsnr_pct": max(map(abs, dsnr)) if dsnr else None,
                           "bf16_dsnr_pct_mean": statistics.fmean(dsnr) if dsnr else None,
                           "bf16_dsnr_pct_sigma": statistics.pstdev(dsnr) if dsnr else None,
                           "bf16_bright_within_3pct": sum(abs(v) <= 3.0 for v in dsnr),
                           "bf16_max_rel_power_err": err_b, "fp32_max_rel_power_err": err_f,
                           "fp8_same_bin_vs_fp64": same_q,
                           "fp8_max_abs_dsnr_pct": max(map(abs, dsnr_q)) if dsnr_q else None,
                           "fp8_dsnr_pct_sigma": statistics.pstdev(dsnr_q) if dsnr_q else None,
                           "fp8_max_rel_power_err": err_q}
        del pl_d

    out["plane_and_peaks"] = {"workload": "the single-DM BF16 plane and its thresholded peaks", **fused_pk}
    if not args.no_series:
        out["series_search"] = series_search_timing(args, cfg, dev, pl_b)

    if not args.no_harmonic:
        out["harmonic_sum"] = {"workload": "the single-DM BF16 plane, BF16 sums out", **harm}

    if not args.no_refine:
        out["refinement"] = refinement_timing(cfg, dev, x, max(10, min(args.steps, 50)))

    if not args.no_jerk:
        out["jerk"] = jerk_volume(args, cfg, dev, x, plane_b)

    if not args.no_prep:
        out["spectrum_preparation"] = prep_timing(args, cfg, dev)

    if not args.no_canopy:
        out["noise_canopy"] = noise_canopy(args, cfg, dev)

    if not args.no_batched:
        out["batched"] = batched_search(args, cfg, dev)

    if not args.no_wide:
        out["wide"] = wide_search(args, dev)

    if not args.no_cpu_baseline:
        r_c = int(round(sp.pulsars[0].r_bar(sp.T)))
        note("timing the FP64 CPU oracle")
        out["cpu_baseline"] = cpu_baseline(sp.spec, cfg, r_c)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
