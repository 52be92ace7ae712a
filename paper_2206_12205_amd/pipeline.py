"""Batched acceleration search over many spectra (dedispersion trials).

Orchestration only: every step runs in libfdas kernels through the C ABI.
Spectra of uneven length share one template grid.  They are grouped into
length classes (powers of two); each class gets the kernel configuration the
autotuner (fdas_tune) measures fastest for its longest member, and its jobs
are packed into chunks whose planes fit one reusable plane buffer.  A pass
over the batch runs, per chunk, fdas_correlate_batch_peaks: one persistent
correlation launch that also flags the peak finder's tiles while it stores
the planes, then one count, scan and write over all of the chunk's planes
(fused=False instead runs fdas_correlate_batch and fdas_peaks on every job's
plane); with harmonics, one fdas_batch_harmonic_sums_peaks call per chunk
then finds the thresholded peaks of every job's sums over its first H
harmonics, for every requested H, without storing the sums.  The full set of
planes (tens of GB in BF16 for hundreds of trials) is never held at once.  A pass issues kernels only, so it can be recorded
once as a HIP graph (capture) and replayed.
"""
from __future__ import annotations

import ctypes
import math

from . import fdas as F


class BatchSearch:
    """Peaks of the f-fdot planes of a batch of packed spectra.

    lengths      bins of each spectrum; spectra are packed back to back in a
                 complex64 device tensor in this order
    buffer_bytes size of the reused plane buffer
    tune         measure the kernel configuration per length class (else the
                 library's defaults)
    harmonics    {H: threshold} for H > 1: the peaks of every job's sum over
                 its first H harmonics are found too (all H and all jobs of a
                 chunk in one fdas_batch_harmonic_sums_peaks call)
    """

    def __init__(self, lengths, z_min, z_step, n_z, n_taps, compute="bf16", plane_dtype="bf16",
                 buffer_bytes=8 << 30, tune=True, tune_reps=3, device="cuda:0", peak_capacity=1 << 12,
                 harmonics=None):
        import torch
        self.lengths = [int(v) for v in lengths]
        if not self.lengths or min(self.lengths) < 1:
            raise ValueError("every spectrum needs at least one bin")
        self.n_z = int(n_z)
        self.device = torch.device(device)
        self.spec_off = [0]
        for v in self.lengths[:-1]:
            self.spec_off.append(self.spec_off[-1] + v)
        self.total_bins = sum(self.lengths)
        self.cells = self.n_z * self.total_bins
        elem = {"bf16": 2, "fp32": 4, "fp64": 8}[plane_dtype]
        self.plane_dtype = plane_dtype
        self.peak_capacity = int(peak_capacity)
        common = dict(z_min=z_min, z_step=z_step, n_z=n_z, n_taps=n_taps, compute=compute,
                      plane_dtype=plane_dtype)
        max_job = max(self.lengths)
        if self.n_z * max_job * elem > buffer_bytes:
            raise ValueError("the plane buffer cannot hold the longest spectrum's plane")
        # length classes: ceil(log2(n))
        classes = {}
        for i, v in enumerate(self.lengths):
            classes.setdefault(max(int(math.ceil(math.log2(v))), 0), []).append(i)
        self.tuned = {}
        self.chunks = []          # (plan, job indices, plane offsets in the buffer, first slot)
        self.slot = [0] * len(self.lengths)   # row of job i in the peak lists (chunk order)
        self._next_slot = 0
        for cls in sorted(classes):
            jobs = classes[cls]
            cmax = max(self.lengths[i] for i in jobs)
            knobs = dict(seg_len=0, algo="auto", z_chunk=0)
            if tune:
                # timed on one spectrum as long as the whole class (capped), so
                # the candidate sees the amount of work of the class's launch
                n_probe = min(sum(self.lengths[i] for i in jobs), max(cmax, 1 << 24))
                probe = torch.randn(n_probe, dtype=torch.complex64, device=self.device,
                                    generator=torch.Generator(device=self.device).manual_seed(cls))
                t = F.tune(probe, max_bins=n_probe, reps=tune_reps, **common)
                knobs = dict(seg_len=t["seg_len"], algo=t["algo"], z_chunk=t["z_chunk"])
                self.tuned[cls] = t
                del probe
            # pack the class's jobs into buffer-sized chunks
            cur, used = [], 0
            for i in jobs:
                need = self.n_z * self.lengths[i] * elem
                if cur and used + need > buffer_bytes:
                    self.chunks.append(self._chunk(cur, cmax, knobs, common))
                    cur, used = [], 0
                cur.append(i)
                used += need
            if cur:
                self.chunks.append(self._chunk(cur, cmax, knobs, common))
        cells_max = max(sum(self.n_z * self.lengths[i] for i in ch[1]) for ch in self.chunks)
        self.buffer = torch.empty(cells_max, dtype=self.chunks[0][0].torch_plane_dtype(), device=self.device)
        self.peaks_raw = torch.empty((len(self.lengths), self.peak_capacity, 24), dtype=torch.uint8,
                                     device=self.device)
        self.n_found = torch.zeros(len(self.lengths), dtype=torch.int64, device=self.device)
        # scratch of the batched peak finder, shared by the chunks (they run in order on one stream)
        need = 0
        for pl, _, _, _ in self.chunks:
            nb = ctypes.c_size_t(0)
            F._check(F.lib().fdas_batch_peaks_workspace(pl._h, ctypes.byref(nb)), "fdas_batch_peaks_workspace")
            need = max(need, nb.value)
        self.peak_scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
        # harmonic sums: per chunk one fdas_batch_harmonic_sums_peaks call (the
        # sums of every job of the chunk, never stored); its lists (level l,
        # job k of the chunk) at list_base[chunk] + l * jobs_in_chunk + k
        self.harmonics = {int(h): float(t) for h, t in (harmonics or {}).items()}
        if any(h < 2 for h in self.harmonics):
            raise ValueError("harmonics are sums over H >= 2 harmonics")
        if self.harmonics:
            hs = sorted(self.harmonics)
            self.list_base, tot, need = [], 0, 0
            for pl, jobs, _, _ in self.chunks:
                self.list_base.append(tot)
                tot += len(hs) * len(jobs)
                need = max(need, pl.batch_sums_peaks_bytes(hs))
            self.hpeaks_all = torch.empty((tot, self.peak_capacity, 24), dtype=torch.uint8, device=self.device)
            self.hn_found_all = torch.zeros(tot, dtype=torch.int64, device=self.device)
            self.sums_scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
            self.chunk_of = {}
            for c, (_, jobs, _, _) in enumerate(self.chunks):
                for k, i in enumerate(jobs):
                    self.chunk_of[i] = (c, k)

    def _chunk(self, jobs, cmax, knobs, common):
        pl = F.Plan(max_bins=cmax, max_jobs=len(jobs), device=self.device, **knobs, **common)
        table = (F.FdasJob * len(jobs))()
        po = 0
        for k, i in enumerate(jobs):
            table[k] = F.FdasJob(self.spec_off[i], self.lengths[i], po)
            po += self.n_z * self.lengths[i]
        F._check(F.lib().fdas_set_batch(pl._h, table, len(jobs), self.total_bins, po, F._stream_ptr(None)),
                 "fdas_set_batch")
        offs = []
        po = 0
        for i in jobs:
            offs.append(po)
            po += self.n_z * self.lengths[i]
        slot0 = self._next_slot
        for k, i in enumerate(jobs):
            self.slot[i] = slot0 + k
        self._next_slot += len(jobs)
        return pl, list(jobs), offs, slot0

    def run(self, spectra, threshold, stream=None, find_peaks=True, fused=True):
        """One pass: planes chunk by chunk into the buffer, peaks of every
        job's plane into the per-job peak lists (asynchronous on stream).
        find_peaks=False runs the correlations only (for timing); fused=False
        finds the peaks with a separate fdas_peaks call per job."""
        import torch
        if spectra.dtype != torch.complex64 or not spectra.is_contiguous() or spectra.numel() < self.total_bins:
            raise ValueError("spectra must be a contiguous complex64 tensor holding every packed spectrum")
        s = F._stream_ptr(stream)
        L = F.lib()
        esz = self.buffer.element_size()
        sp = ctypes.c_void_p(spectra.data_ptr())
        buf = ctypes.c_void_p(self.buffer.data_ptr())
        for c, (pl, jobs, offs, slot0) in enumerate(self.chunks):
            if find_peaks and fused:
                F._check(L.fdas_correlate_batch_peaks(
                    pl._h, sp, buf, float(threshold), ctypes.c_void_p(self.peaks_raw[slot0].data_ptr()),
                    self.peak_capacity, ctypes.c_void_p(self.n_found[slot0:slot0 + 1].data_ptr()),
                    ctypes.c_void_p(self.peak_scratch.data_ptr()), self.peak_scratch.numel(), s),
                    "fdas_correlate_batch_peaks")
            else:
                F._check(L.fdas_correlate_batch(pl._h, sp, buf, s), "fdas_correlate_batch")
                for k, (i, po) in enumerate(zip(jobs, offs) if find_peaks else ()):
                    F._check(L.fdas_peaks(pl._h, ctypes.c_void_p(self.buffer.data_ptr() + po * esz),
                                          self.lengths[i], float(threshold),
                                          ctypes.c_void_p(self.peaks_raw[slot0 + k].data_ptr()), self.peak_capacity,
                                          ctypes.c_void_p(self.n_found[slot0 + k:].data_ptr()), s),
                             "fdas_peaks")
            if not find_peaks or not self.harmonics:
                continue
            hs = sorted(self.harmonics)
            lb = self.list_base[c]
            pl.batch_sums_peaks_async(self.buffer.data_ptr(), hs, [self.harmonics[h] for h in hs],
                                      self.hpeaks_all[lb].data_ptr(), self.peak_capacity,
                                      self.hn_found_all[lb:].data_ptr(), self.sums_scratch, stream)

    def capture(self, spectra, threshold, find_peaks=True, fused=True):
        """Record one pass (run) into a HIP graph and return it
        (torch.cuda.CUDAGraph).  Every launch of a pass has fixed arguments
        (each chunk has its own plan and job table, set at construction), and
        the library records only kernels (counters and peak counts are
        cleared by kernels, not memsets), so g.replay() runs a whole pass on
        the current contents of spectra and refreshes the peak lists."""
        import torch
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.run(spectra, threshold, find_peaks=find_peaks, fused=fused)   # warm-up on the capture stream
        torch.cuda.current_stream(self.device).wait_stream(side)
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(spectra, threshold, find_peaks=find_peaks, fused=fused)
        return g

    def peaks(self, i, H=1, truncate=False):
        """Peak list of job i after run() (host copy): dict of z_idx, r, power,
        n_found; H > 1: the peaks of its sum over H harmonics.  A list that
        overflowed peak_capacity raises fdas.PeakCapacityError (its first
        entries and true count in the error's result) unless truncate is set."""
        import numpy as np
        if H == 1:
            raw_all, nf, row = self.peaks_raw, self.n_found, self.slot[i]
        else:
            c, k = self.chunk_of[i]
            lvl = sorted(self.harmonics).index(H)
            raw_all, nf = self.hpeaks_all, self.hn_found_all
            row = self.list_base[c] + lvl * len(self.chunks[c][1]) + k
        found = int(nf[row].item())
        k = min(found, self.peak_capacity)
        raw = raw_all[row, :k].cpu().numpy()
        rec = raw.view(np.dtype([("r", "<i8"), ("z_idx", "<i4"), ("job", "<i4"),
                                 ("power", "<f4"), ("reserved", "<f4")])).reshape(-1)
        res = {"z_idx": rec["z_idx"].copy(), "r": rec["r"].copy(), "power": rec["power"].copy(),
               "n_found": found, "truncated": found > self.peak_capacity}
        if res["truncated"] and not truncate:
            raise F.PeakCapacityError(f"job {i} peaks (H = {H})", res)
        return res


def search_series(plan, series, threshold, harmonics=(1, 2, 4, 8, 16), capacity=1 << 16, stream=None):
    """One dedispersed time series through the whole search on the GPU.

    series     contiguous float32 device tensor, a power-of-two length n_t
    plan       a fdas.Plan whose max_bins covers n_t / 2
    threshold  a float, or a dict H -> float (noise powers of a sum of H
               normalised powers have mean H)
    Steps: the normalised spectrum (fdas_prepare), the plane with its
    thresholded peaks (fdas_correlate_peaks), and the thresholded peaks of
    every sum over H > 1 harmonics in one summing pass, the sums themselves
    not stored (fdas_harmonic_peaks: the same lists as
    fdas_harmonic_sums_peaks).  Returns (spectrum, plane, {H: peaks dict}).
    """
    spec = F.prepare(series, stream=stream)
    thr = (lambda h: float(threshold[h])) if isinstance(threshold, dict) else (lambda h: float(threshold))
    plane, pk1 = plan.correlate_peaks(spec, thr(1), capacity=capacity, stream=stream)
    found = {1: pk1} if 1 in harmonics else {}
    hs = sorted(h for h in set(harmonics) if h > 1)
    if hs:
        lists = plan.harmonic_peaks(plane, hs, [thr(h) for h in hs], capacity=capacity, stream=stream)
        found.update(zip(hs, lists))
    return spec, plane, found
