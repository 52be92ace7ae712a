"""Python binding of libfdas (ctypes).  Argument marshalling only: every step
of the hot path runs in the library's HIP kernels; PyTorch provides device
memory and streams.  The names follow the C ABI in include/fdas.h.

Loading fails loudly when the HIP library has not been built (there is no
fallback of any kind).
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdas.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fdas.h")

FP32, BF16, FP8E4M3, FP64 = 0, 1, 2, 3
DTYPES = {"fp32": FP32, "bf16": BF16, "fp8": FP8E4M3, "fp64": FP64}
ALGO_AUTO, ALGO_VALU, ALGO_MFMA = 0, 1, 2
ALGOS = {"auto": ALGO_AUTO, "valu": ALGO_VALU, "mfma": ALGO_MFMA}

OK, E_INVALID, E_WORKSPACE, E_HIP, E_CAPACITY, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5, -6
# size of the fixed per-GPU scratch array behind fdas_harmonic_sums_peaks_noalloc
NOALLOC_SCRATCH_BYTES = 8 << 20


class FdasConfig(ctypes.Structure):
    _fields_ = [("max_bins", ctypes.c_int64), ("z_min", ctypes.c_double),
                ("z_step", ctypes.c_double), ("n_z", ctypes.c_int32),
                ("n_taps", ctypes.c_int32), ("seg_len", ctypes.c_int32),
                ("compute", ctypes.c_int32), ("plane_dtype", ctypes.c_int32),
                ("z_chunk", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("max_jobs", ctypes.c_int32)]


class FdasJob(ctypes.Structure):
    _fields_ = [("spec_off", ctypes.c_int64), ("n_bins", ctypes.c_int64),
                ("plane_off", ctypes.c_int64)]


class FdasPeak(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int64), ("z_idx", ctypes.c_int32), ("job", ctypes.c_int32),
                ("power", ctypes.c_float), ("reserved", ctypes.c_float)]


class FdasLayout(ctypes.Structure):
    _fields_ = [("total_bytes", ctypes.c_size_t), ("bank_offset", ctypes.c_size_t),
                ("bank_bytes", ctypes.c_size_t), ("twiddle_offset", ctypes.c_size_t),
                ("twiddle_bytes", ctypes.c_size_t), ("scratch_offset", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t), ("seg_len", ctypes.c_int32),
                ("valid_per_seg", ctypes.c_int32), ("z_chunk", ctypes.c_int32),
                ("bank_elem_bytes", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("tables_offset", ctypes.c_size_t), ("tables_bytes", ctypes.c_size_t)]


class FdasError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = lib().fdas_strerror(status).decode()
        if status == E_HIP:
            msg += f" (hip error {lib().fdas_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{status}]")
        self.status = status


class PeakCapacityError(FdasError):
    """FDAS_E_CAPACITY: a peak list overflowed.  `result` holds what the call
    would have returned (every list with its first `capacity` peaks and its
    true n_found, flagged truncated)."""

    def __init__(self, what: str, result):
        super().__init__(E_CAPACITY, what)
        self.result = result


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfdas.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2206_12205_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.fdas_plan.argtypes = [ctypes.POINTER(FdasConfig), ctypes.POINTER(P),
                                ctypes.POINTER(ctypes.c_size_t)]
        L.fdas_plan.restype = ctypes.c_int
        L.fdas_destroy.argtypes = [P]
        L.fdas_destroy.restype = None
        L.fdas_set_workspace.argtypes = [P, P, ctypes.c_size_t]
        L.fdas_get_layout.argtypes = [P, ctypes.POINTER(FdasLayout)]
        L.fdas_make_templates.argtypes = [P, P]
        L.fdas_correlate.argtypes = [P, P, I64, P, P]
        L.fdas_tune_workspace.argtypes = [ctypes.POINTER(FdasConfig), ctypes.POINTER(ctypes.c_size_t)]
        L.fdas_tune.argtypes = [ctypes.POINTER(FdasConfig), P, I64, P, P, ctypes.c_size_t, I32,
                                ctypes.POINTER(FdasConfig), ctypes.POINTER(ctypes.c_float), P]
        L.fdas_set_batch.argtypes = [P, ctypes.POINTER(FdasJob), I32, I64, I64, P]
        L.fdas_correlate_batch.argtypes = [P, P, P, P]
        L.fdas_peaks.argtypes = [P, P, I64, ctypes.c_float, P, I64, P, P]
        L.fdas_correlate_peaks.argtypes = [P, P, I64, P, ctypes.c_float, P, I64, P, P]
        L.fdas_batch_peaks_workspace.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.fdas_correlate_batch_peaks.argtypes = [P, P, P, ctypes.c_float, P, I64, P, P, ctypes.c_size_t, P]
        L.fdas_harmonic_sum.argtypes = [P, P, I64, I32, P, P]
        L.fdas_harmonic_sum_peaks.argtypes = [P, P, I64, I32, P, ctypes.c_float, P, I64, P, P]
        L.fdas_harmonic_sums.argtypes = [P, P, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(P), P]
        L.fdas_harmonic_sums_peaks_workspace.argtypes = [P, I64, I32, ctypes.POINTER(I32),
                                                         ctypes.POINTER(ctypes.c_size_t)]
        L.fdas_harmonic_sums_peaks.argtypes = [P, P, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(P),
                                               ctypes.POINTER(ctypes.c_float), ctypes.POINTER(P), I64, P, P,
                                               ctypes.c_size_t, P]
        L.fdas_harmonic_sums_peaks_noalloc.argtypes = [P, P, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(P),
                                                       ctypes.POINTER(ctypes.c_float), ctypes.POINTER(P), I64, P,
                                                       P]
        L.fdas_batch_harmonic_sums_peaks_workspace.argtypes = [P, I32, ctypes.POINTER(I32),
                                                               ctypes.POINTER(ctypes.c_size_t)]
        L.fdas_batch_harmonic_sums_peaks.argtypes = [P, P, I32, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_float),
                                                     P, I64, P, P, ctypes.c_size_t, P]
        L.fdas_harmonic_peaks_workspace.argtypes = [P, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_size_t)]
        L.fdas_harmonic_peaks.argtypes = [P, P, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_float), P, I64,
                                          P, P, ctypes.c_size_t, P]
        L.fdas_band_max.argtypes = [P, P, I64, P, I32, P, P]
        L.fdas_prepare_workspace.argtypes = [I64, ctypes.POINTER(ctypes.c_size_t)]
        L.fdas_prepare.argtypes = [P, I64, P, P, ctypes.c_size_t, P]
        D = ctypes.c_double
        L.fdas_make_templates_jerk.argtypes = [P, D, P]
        L.fdas_refine.argtypes = [P, I64, I32, P, P, P, P, P, I32, I32, D, D, P]
        L.fdas_refine_backward.argtypes = [P, I64, I32, P, P, P, P, P, I32, P]
        L.fdas_peaks_check.argtypes = [P, I32, I64, ctypes.POINTER(I64), P]
        L.fdas_strerror.argtypes = [ctypes.c_int]
        L.fdas_strerror.restype = ctypes.c_char_p
        L.fdas_last_hip_error.restype = ctypes.c_int
        L.fdas_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions include/fdas.h declares."""
    with open(HEADER) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fdas_[a-z_]+)\s*\(", txt)))


def _check(status: int, what: str):
    if status != OK:
        raise FdasError(status, what)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_config(max_bins, z_min, z_step, n_z, n_taps, seg_len=0, compute="fp32",
                plane_dtype=None, z_chunk=0, algo="auto", max_jobs=0) -> FdasConfig:
    c = DTYPES[compute] if isinstance(compute, str) else int(compute)
    if plane_dtype is None:
        plane_dtype = {FP32: FP32, BF16: BF16, FP64: FP64}.get(c, FP32)
    pd = DTYPES[plane_dtype] if isinstance(plane_dtype, str) else int(plane_dtype)
    a = ALGOS[algo] if isinstance(algo, str) else int(algo)
    return FdasConfig(int(max_bins), float(z_min), float(z_step), int(n_z), int(n_taps),
                      int(seg_len), c, pd, int(z_chunk), a, int(max_jobs))


def peak_counts(n_found, n_lists, capacity, stream=None):
    """True counts of n_lists peak lists (fdas_peaks_check: waits for the
    stream, copies the device counts) -> (list of counts, overflowed)."""
    counts = (ctypes.c_int64 * int(n_lists))()
    st = lib().fdas_peaks_check(ctypes.c_void_p(n_found.data_ptr()), int(n_lists), int(capacity), counts,
                                _stream_ptr(stream))
    if st not in (OK, E_CAPACITY):
        raise FdasError(st, "fdas_peaks_check")
    return [int(v) for v in counts], st == E_CAPACITY


def _capacity_result(what, overflowed, truncate, result):
    if overflowed and not truncate:
        raise PeakCapacityError(what, result)
    return result


def peak_records(raw, found, capacity):
    """Peak records (a (capacity, 24) uint8 tensor of fdas_peak entries) ->
    dict of numpy arrays z_idx, r, power, job, the true count n_found and
    truncated (more peaks than capacity: the list holds the first ones; the
    C calls cannot tell without a device synchronisation, the wrapper can)."""
    import numpy as np
    k = min(int(found), int(capacity))
    rec = raw[:k].cpu().numpy().view(np.dtype([("r", "<i8"), ("z_idx", "<i4"), ("job", "<i4"),
                                              ("power", "<f4"), ("reserved", "<f4")])).reshape(-1)
    return {"z_idx": rec["z_idx"].copy(), "r": rec["r"].copy(), "power": rec["power"].copy(),
            "job": rec["job"].copy(), "n_found": int(found), "truncated": int(found) > int(capacity)}


class Plan:
    """An FDAS plan with its device workspace (a torch uint8 tensor)."""

    def __init__(self, max_bins, z_min, z_step, n_z, n_taps, seg_len=0,
                 compute="fp32", plane_dtype=None, z_chunk=0, device="cuda:0",
                 make_templates=True, algo="auto", max_jobs=0):
        import torch
        self.cfg = make_config(max_bins, z_min, z_step, n_z, n_taps, seg_len, compute,
                               plane_dtype, z_chunk, algo, max_jobs)
        h = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        _check(lib().fdas_plan(ctypes.byref(self.cfg), ctypes.byref(h), ctypes.byref(nbytes)),
               "fdas_plan")
        self._h = h
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        _check(lib().fdas_set_workspace(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                        self.workspace.numel()), "fdas_set_workspace")
        self.layout = FdasLayout()
        _check(lib().fdas_get_layout(self._h, ctypes.byref(self.layout)), "fdas_get_layout")
        self.n_z = int(n_z)
        self.plane_dtype = self.cfg.plane_dtype
        if make_templates:
            self.make_templates()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fdas_destroy(h)
            self._h = None

    @property
    def seg_len(self) -> int:
        return int(self.layout.seg_len)

    @property
    def algo(self) -> str:
        return {ALGO_VALU: "valu", ALGO_MFMA: "mfma"}[int(self.layout.algo)]

    def make_templates(self, stream=None, w=0.0):
        """Template bank of the plan's z grid; w != 0: the plane of jerk w
        (fdas_make_templates_jerk)."""
        if w == 0.0:
            _check(lib().fdas_make_templates(self._h, _stream_ptr(stream)), "fdas_make_templates")
        else:
            _check(lib().fdas_make_templates_jerk(self._h, float(w), _stream_ptr(stream)),
                   "fdas_make_templates_jerk")

    def torch_plane_dtype(self):
        import torch
        return {FP32: torch.float32, BF16: torch.bfloat16, FP64: torch.float64}[self.plane_dtype]

    def empty_plane(self, n_bins):
        import torch
        return torch.empty((self.n_z, int(n_bins)), dtype=self.torch_plane_dtype(),
                           device=self.device)

    def correlate(self, spectrum, plane=None, stream=None):
        """f-fdot plane of a complex64 device spectrum -> (n_z, N) tensor."""
        import torch
        if spectrum.dtype != torch.complex64 or not spectrum.is_contiguous():
            raise ValueError("spectrum must be a contiguous complex64 tensor")
        n = spectrum.numel()
        if plane is None:
            plane = self.empty_plane(n)
        if plane.dtype != self.torch_plane_dtype() or tuple(plane.shape) != (self.n_z, n) \
                or not plane.is_contiguous():
            raise ValueError("plane has the wrong dtype, shape or layout")
        _check(lib().fdas_correlate(self._h, ctypes.c_void_p(spectrum.data_ptr()), n,
                                    ctypes.c_void_p(plane.data_ptr()), _stream_ptr(stream)),
               "fdas_correlate")
        return plane

    def set_batch(self, lengths, spectra_bins=None, plane_cells=None, stream=None):
        """Store a batch of spectra packed back to back (job i: lengths[i] bins
        at the running offset, its plane at n_z times that offset).  Returns
        the (spec_off, plane_off) lists."""
        lengths = [int(v) for v in lengths]
        jobs = (FdasJob * max(len(lengths), 1))()
        so, po, offs = 0, 0, []
        for i, nb in enumerate(lengths):
            jobs[i] = FdasJob(so, nb, po)
            offs.append((so, po))
            so += nb
            po += self.n_z * nb
        self.batch_lengths = lengths
        self.batch_offsets = offs
        self.batch_bins = so if spectra_bins is None else int(spectra_bins)
        self.batch_cells = po if plane_cells is None else int(plane_cells)
        _check(lib().fdas_set_batch(self._h, jobs, len(lengths), self.batch_bins, self.batch_cells,
                                    _stream_ptr(stream)), "fdas_set_batch")
        return offs

    def correlate_batch(self, spectra, planes=None, stream=None):
        """Planes of the stored batch: spectra is the packed complex64 device
        tensor, planes a flat tensor of the plane dtype (allocated if None)."""
        import torch
        if spectra.dtype != torch.complex64 or not spectra.is_contiguous() \
                or spectra.numel() < self.batch_bins:
            raise ValueError("spectra must be a contiguous complex64 tensor of the batch's size")
        if planes is None:
            planes = torch.empty(self.batch_cells, dtype=self.torch_plane_dtype(), device=self.device)
        if planes.dtype != self.torch_plane_dtype() or not planes.is_contiguous() \
                or planes.numel() < self.batch_cells:
            raise ValueError("planes has the wrong dtype, size or layout")
        _check(lib().fdas_correlate_batch(self._h, ctypes.c_void_p(spectra.data_ptr()),
                                          ctypes.c_void_p(planes.data_ptr()), _stream_ptr(stream)),
               "fdas_correlate_batch")
        return planes

    def batch_plane(self, planes, i):
        """(n_z, n_i) view of job i's plane inside the flat batch planes."""
        nb = self.batch_lengths[i]
        po = self.batch_offsets[i][1]
        return planes[po:po + self.n_z * nb].view(self.n_z, nb)

    def peaks(self, plane, threshold, capacity=1 << 16, stream=None, truncate=False):
        """Peaks of a plane -> dict of numpy arrays z_idx, r, power and n_found.
        More peaks than capacity raises PeakCapacityError (the first ones and
        the true count in its result) unless truncate is set."""
        import torch
        n = plane.shape[1]
        out = torch.empty((max(int(capacity), 1), 24), dtype=torch.uint8, device=self.device)
        nf = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().fdas_peaks(self._h, ctypes.c_void_p(plane.data_ptr()), n,
                                float(threshold), ctypes.c_void_p(out.data_ptr()),
                                int(capacity), ctypes.c_void_p(nf.data_ptr()),
                                _stream_ptr(stream)), "fdas_peaks")
        (found,), over = peak_counts(nf, 1, capacity, stream)
        return _capacity_result("fdas_peaks", over, truncate, peak_records(out, found, capacity))

    def correlate_peaks(self, spectrum, threshold, capacity=1 << 16, plane=None, stream=None, truncate=False):
        """Plane and thresholded peaks of a spectrum in one call
        (fdas_correlate_peaks) -> (plane, peaks dict as from peaks());
        overflow as for peaks()."""
        import torch
        if spectrum.dtype != torch.complex64 or not spectrum.is_contiguous():
            raise ValueError("spectrum must be a contiguous complex64 tensor")
        n = spectrum.numel()
        if plane is None:
            plane = self.empty_plane(n)
        if plane.dtype != self.torch_plane_dtype() or tuple(plane.shape) != (self.n_z, n) \
                or not plane.is_contiguous():
            raise ValueError("plane has the wrong dtype, shape or layout")
        out = torch.empty((max(int(capacity), 1), 24), dtype=torch.uint8, device=self.device)
        nf = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().fdas_correlate_peaks(self._h, ctypes.c_void_p(spectrum.data_ptr()), n,
                                          ctypes.c_void_p(plane.data_ptr()), float(threshold),
                                          ctypes.c_void_p(out.data_ptr()), int(capacity),
                                          ctypes.c_void_p(nf.data_ptr()), _stream_ptr(stream)),
               "fdas_correlate_peaks")
        (found,), over = peak_counts(nf, 1, capacity, stream)
        return _capacity_result("fdas_correlate_peaks", over, truncate,
                                (plane, peak_records(out, found, capacity)))

    def batch_peaks_scratch(self):
        """Device scratch for fdas_correlate_batch_peaks on the stored batch
        (a uint8 tensor, reused while large enough)."""
        import torch
        nb = ctypes.c_size_t(0)
        _check(lib().fdas_batch_peaks_workspace(self._h, ctypes.byref(nb)), "fdas_batch_peaks_workspace")
        cur = getattr(self, "_batch_scratch", None)
        if cur is None or cur.numel() < nb.value:
            cur = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=self.device)
            self._batch_scratch = cur
        return cur

    def correlate_batch_peaks_async(self, spectra, planes, threshold, out, n_found, stream=None):
        """Enqueue fdas_correlate_batch_peaks: out a (n_jobs, capacity, 24)
        uint8 device tensor of peak records, n_found an int64 device tensor
        of n_jobs counts.  No host synchronisation (graph-capturable)."""
        import torch
        if spectra.dtype != torch.complex64 or not spectra.is_contiguous() \
                or spectra.numel() < self.batch_bins:
            raise ValueError("spectra must be a contiguous complex64 tensor of the batch's size")
        if planes.dtype != self.torch_plane_dtype() or not planes.is_contiguous() \
                or planes.numel() < self.batch_cells:
            raise ValueError("planes has the wrong dtype, size or layout")
        n_jobs = len(self.batch_lengths)
        if out.dim() != 3 or out.shape[0] != n_jobs or out.shape[2] != 24 or out.dtype != torch.uint8 \
                or not out.is_contiguous() or n_found.numel() < n_jobs or n_found.dtype != torch.int64:
            raise ValueError("out must be (n_jobs, capacity, 24) uint8, n_found n_jobs int64")
        scr = self.batch_peaks_scratch()
        _check(lib().fdas_correlate_batch_peaks(self._h, ctypes.c_void_p(spectra.data_ptr()),
                                                ctypes.c_void_p(planes.data_ptr()), float(threshold),
                                                ctypes.c_void_p(out.data_ptr()), int(out.shape[1]),
                                                ctypes.c_void_p(n_found.data_ptr()),
                                                ctypes.c_void_p(scr.data_ptr()), scr.numel(),
                                                _stream_ptr(stream)), "fdas_correlate_batch_peaks")

    def correlate_batch_peaks(self, spectra, threshold, capacity=1 << 12, planes=None, stream=None,
                              truncate=False):
        """Planes of the stored batch and every job's peaks
        (fdas_correlate_batch_peaks) -> (planes, list of peaks dicts);
        overflow of any job's list as for peaks()."""
        import torch
        if planes is None:
            planes = torch.empty(self.batch_cells, dtype=self.torch_plane_dtype(), device=self.device)
        n_jobs = len(self.batch_lengths)
        out = torch.empty((n_jobs, max(int(capacity), 1), 24), dtype=torch.uint8, device=self.device)
        nf = torch.zeros(n_jobs, dtype=torch.int64, device=self.device)
        self.correlate_batch_peaks_async(spectra, planes, threshold, out, nf, stream)
        found, over = peak_counts(nf, n_jobs, capacity, stream)
        return _capacity_result("fdas_correlate_batch_peaks", over, truncate,
                                (planes, [peak_records(out[i], found[i], capacity) for i in range(n_jobs)]))

    def band_max(self, plane, windows, stream=None):
        """Highest cell of each window (z_lo, z_hi, r_lo, r_hi) of a plane
        (fdas_band_max) -> dict of numpy arrays z_idx, r, power."""
        import numpy as np
        import torch
        if plane.dim() != 2 or plane.shape[0] != self.n_z or plane.dtype != self.torch_plane_dtype() \
                or not plane.is_contiguous():
            raise ValueError("plane must be a contiguous (n_z, n) tensor of the plan's plane dtype")
        win = torch.as_tensor(np.asarray(windows, dtype=np.int64).reshape(-1, 4), device=self.device).contiguous()
        out = torch.empty((win.shape[0], 24), dtype=torch.uint8, device=self.device)
        _check(lib().fdas_band_max(self._h, ctypes.c_void_p(plane.data_ptr()), plane.shape[1],
                                   ctypes.c_void_p(win.data_ptr()), int(win.shape[0]),
                                   ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "fdas_band_max")
        rec = out.cpu().numpy().view(np.dtype([("r", "<i8"), ("z_idx", "<i4"), ("job", "<i4"),
                                              ("power", "<f4"), ("reserved", "<f4")])).reshape(-1)
        return {"z_idx": rec["z_idx"].astype(np.int64), "r": rec["r"].copy(), "power": rec["power"].copy()}

    def harmonic_sum(self, plane, n_harm, out=None, stream=None):
        """Incoherent sum of the first n_harm harmonics of a plane (fdas_harmonic_sum):
        an (n_z, (n - 1) // n_harm + 1) tensor of the plane dtype."""
        import torch
        if plane.dim() != 2 or plane.shape[0] != self.n_z or plane.dtype != self.torch_plane_dtype() \
                or not plane.is_contiguous():
            raise ValueError("plane must be a contiguous (n_z, n) tensor of the plan's plane dtype")
        n = plane.shape[1]
        nh = (n - 1) // int(n_harm) + 1 if n > 0 else 0
        if out is None:
            out = torch.empty((self.n_z, nh), dtype=plane.dtype, device=self.device)
        elif out.shape != (self.n_z, nh) or out.dtype != plane.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous (n_z, N_H) tensor of the plane dtype")
        _check(lib().fdas_harmonic_sum(self._h, ctypes.c_void_p(plane.data_ptr()), n, int(n_harm),
                                       ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "fdas_harmonic_sum")
        return out

    def harmonic_sums(self, plane, n_harms, outs=None, stream=None):
        """Sums for an increasing list of harmonic counts in one pass
        (fdas_harmonic_sums) -> list of (n_z, (n - 1) // H + 1) tensors."""
        import torch
        if plane.dim() != 2 or plane.shape[0] != self.n_z or plane.dtype != self.torch_plane_dtype() \
                or not plane.is_contiguous():
            raise ValueError("plane must be a contiguous (n_z, n) tensor of the plan's plane dtype")
        n = plane.shape[1]
        hs = [int(h) for h in n_harms]
        if outs is None:
            outs = [torch.empty((self.n_z, (n - 1) // h + 1), dtype=plane.dtype, device=self.device) for h in hs]
        for h, o in zip(hs, outs):
            if o.dtype != plane.dtype or tuple(o.shape) != (self.n_z, (n - 1) // h + 1) or not o.is_contiguous():
                raise ValueError("an output has the wrong dtype, shape or layout")
        harr = (ctypes.c_int32 * len(hs))(*hs)
        parr = (ctypes.c_void_p * len(hs))(*[o.data_ptr() for o in outs])
        _check(lib().fdas_harmonic_sums(self._h, ctypes.c_void_p(plane.data_ptr()), n, len(hs), harr, parr,
                                        _stream_ptr(stream)), "fdas_harmonic_sums")
        return outs

    def harmonic_sums_peaks_async(self, plane, n, n_harms, thresholds, outs, peaks, n_found, scratch,
                                  stream=None):
        """Enqueue fdas_harmonic_sums_peaks on raw device pointers: plane (an
        n-bin plane), outs and peaks lists of device pointers, n_found a
        device pointer to len(n_harms) int64, scratch a uint8 tensor of
        harmonic_sums_peaks_bytes.  No host synchronisation."""
        hs = [int(h) for h in n_harms]
        harr = (ctypes.c_int32 * len(hs))(*hs)
        oarr = (ctypes.c_void_p * len(hs))(*outs)
        tarr = (ctypes.c_float * len(hs))(*[float(t) for t in thresholds])
        parr = (ctypes.c_void_p * len(hs))(*[p for p, _ in peaks])
        cap = peaks[0][1]
        _check(lib().fdas_harmonic_sums_peaks(self._h, ctypes.c_void_p(plane), int(n), len(hs), harr, oarr, tarr,
                                              parr, int(cap), ctypes.c_void_p(n_found),
                                              ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                                              _stream_ptr(stream)), "fdas_harmonic_sums_peaks")

    def harmonic_sums_peaks_noalloc_async(self, plane, n, n_harms, thresholds, outs, peaks, n_found, stream=None):
        """Enqueue fdas_harmonic_sums_peaks_noalloc on raw device pointers
        (arguments as for harmonic_sums_peaks_async, without the scratch: the
        library's fixed per-GPU array serves instead).  Allocates nothing."""
        hs = [int(h) for h in n_harms]
        harr = (ctypes.c_int32 * len(hs))(*hs)
        oarr = (ctypes.c_void_p * len(hs))(*outs)
        tarr = (ctypes.c_float * len(hs))(*[float(t) for t in thresholds])
        parr = (ctypes.c_void_p * len(hs))(*[p for p, _ in peaks])
        cap = peaks[0][1]
        _check(lib().fdas_harmonic_sums_peaks_noalloc(self._h, ctypes.c_void_p(plane), int(n), len(hs), harr, oarr,
                                                      tarr, parr, int(cap), ctypes.c_void_p(n_found),
                                                      _stream_ptr(stream)), "fdas_harmonic_sums_peaks_noalloc")

    def batch_sums_peaks_bytes(self, n_harms):
        """Scratch bytes of fdas_batch_harmonic_sums_peaks for the stored batch."""
        hs = [int(h) for h in n_harms]
        nb = ctypes.c_size_t(0)
        _check(lib().fdas_batch_harmonic_sums_peaks_workspace(self._h, len(hs), (ctypes.c_int32 * len(hs))(*hs),
                                                              ctypes.byref(nb)),
               "fdas_batch_harmonic_sums_peaks_workspace")
        return nb.value

    def batch_sums_peaks_async(self, planes_ptr, n_harms, thresholds, peaks_ptr, capacity, n_found_ptr, scratch,
                               stream=None):
        """Enqueue fdas_batch_harmonic_sums_peaks on raw device pointers:
        peaks_ptr holds n_levels x n_jobs x capacity records, n_found_ptr
        n_levels x n_jobs int64, scratch a uint8 tensor of
        batch_sums_peaks_bytes.  No host synchronisation."""
        hs = [int(h) for h in n_harms]
        harr = (ctypes.c_int32 * len(hs))(*hs)
        tarr = (ctypes.c_float * len(hs))(*[float(t) for t in thresholds])
        _check(lib().fdas_batch_harmonic_sums_peaks(self._h, ctypes.c_void_p(planes_ptr), len(hs), harr, tarr,
                                                    ctypes.c_void_p(peaks_ptr), int(capacity),
                                                    ctypes.c_void_p(n_found_ptr), ctypes.c_void_p(scratch.data_ptr()),
                                                    scratch.numel(), _stream_ptr(stream)),
               "fdas_batch_harmonic_sums_peaks")

    def batch_sums_peaks(self, planes, n_harms, thresholds, capacity=1 << 12, stream=None, truncate=False):
        """Peaks of every job's harmonic sums of the stored batch
        (fdas_batch_harmonic_sums_peaks) -> list over levels of lists over
        jobs of peaks dicts; overflow of any list as for peaks()."""
        import torch
        hs = [int(h) for h in n_harms]
        n_jobs = len(self.batch_offsets)
        pk = torch.empty((len(hs), n_jobs, max(int(capacity), 1), 24), dtype=torch.uint8, device=self.device)
        nf = torch.zeros((len(hs), n_jobs), dtype=torch.int64, device=self.device)
        scr = torch.empty(max(self.batch_sums_peaks_bytes(hs), 1), dtype=torch.uint8, device=self.device)
        self.batch_sums_peaks_async(planes.data_ptr(), hs, thresholds, pk.data_ptr(), capacity, nf.data_ptr(), scr,
                                    stream)
        found, over = peak_counts(nf, len(hs) * n_jobs, capacity, stream)
        res = [[peak_records(pk[l, i], found[l * n_jobs + i], capacity) for i in range(n_jobs)]
               for l in range(len(hs))]
        return _capacity_result("fdas_batch_harmonic_sums_peaks", over, truncate, res)

    def harmonic_sums_peaks_bytes(self, n, n_harms):
        hs = [int(h) for h in n_harms]
        nb = ctypes.c_size_t(0)
        _check(lib().fdas_harmonic_sums_peaks_workspace(self._h, int(n), len(hs), (ctypes.c_int32 * len(hs))(*hs),
                                                        ctypes.byref(nb)), "fdas_harmonic_sums_peaks_workspace")
        return nb.value

    def harmonic_sums_peaks(self, plane, n_harms, thresholds, capacity=1 << 16, stream=None, truncate=False):
        """Several harmonic sums in one pass with the thresholded peaks of
        each (fdas_harmonic_sums_peaks) -> (list of sums, list of peaks
        dicts); overflow of any list as for peaks()."""
        import torch
        if plane.dim() != 2 or plane.shape[0] != self.n_z or plane.dtype != self.torch_plane_dtype() \
                or not plane.is_contiguous():
            raise ValueError("plane must be a contiguous (n_z, n) tensor of the plan's plane dtype")
        n = plane.shape[1]
        hs = [int(h) for h in n_harms]
        outs = [torch.empty((self.n_z, (n - 1) // h + 1), dtype=plane.dtype, device=self.device) for h in hs]
        # each level's list starts 16-byte aligned: an even number of 24-byte records apart
        stride = max(int(capacity), 1)
        stride += stride & 1
        pk = torch.empty((len(hs), stride, 24), dtype=torch.uint8, device=self.device)
        nf = torch.zeros(len(hs), dtype=torch.int64, device=self.device)
        scr = torch.empty(max(self.harmonic_sums_peaks_bytes(n, hs), 1), dtype=torch.uint8, device=self.device)
        self.harmonic_sums_peaks_async(plane.data_ptr(), n, hs, thresholds, [o.data_ptr() for o in outs],
                                       [(pk[l].data_ptr(), int(capacity)) for l in range(len(hs))], nf.data_ptr(),
                                       scr, stream)
        found, over = peak_counts(nf, len(hs), capacity, stream)
        return _capacity_result("fdas_harmonic_sums_peaks", over, truncate,
                                (outs, [peak_records(pk[l], found[l], capacity) for l in range(len(hs))]))

    def harmonic_peaks_bytes(self, n, n_harms):
        """Scratch bytes of fdas_harmonic_peaks for an n-bin plane."""
        hs = [int(h) for h in n_harms]
        nb = ctypes.c_size_t(0)
        _check(lib().fdas_harmonic_peaks_workspace(self._h, int(n), len(hs), (ctypes.c_int32 * len(hs))(*hs),
                                                   ctypes.byref(nb)), "fdas_harmonic_peaks_workspace")
        return nb.value

    def harmonic_peaks_async(self, plane_ptr, n, n_harms, thresholds, peaks_ptr, capacity, n_found_ptr, scratch,
                             stream=None):
        """Enqueue fdas_harmonic_peaks on raw device pointers: peaks_ptr holds
        len(n_harms) x capacity records, n_found_ptr len(n_harms) int64,
        scratch a uint8 tensor of harmonic_peaks_bytes.  No host
        synchronisation."""
        hs = [int(h) for h in n_harms]
        harr = (ctypes.c_int32 * len(hs))(*hs)
        tarr = (ctypes.c_float * len(hs))(*[float(t) for t in thresholds])
        _check(lib().fdas_harmonic_peaks(self._h, ctypes.c_void_p(plane_ptr), int(n), len(hs), harr, tarr,
                                         ctypes.c_void_p(peaks_ptr), int(capacity), ctypes.c_void_p(n_found_ptr),
                                         ctypes.c_void_p(scratch.data_ptr()), scratch.numel(), _stream_ptr(stream)),
               "fdas_harmonic_peaks")

    def harmonic_peaks(self, plane, n_harms, thresholds, capacity=1 << 16, stream=None, truncate=False):
        """The thresholded peaks of several harmonic sums of one plane, the
        sums never stored (fdas_harmonic_peaks) -> list of peaks dicts, one
        per level; overflow of any list as for peaks()."""
        import torch
        if plane.dim() != 2 or plane.shape[0] != self.n_z or plane.dtype != self.torch_plane_dtype() \
                or not plane.is_contiguous():
            raise ValueError("plane must be a contiguous (n_z, n) tensor of the plan's plane dtype")
        n = plane.shape[1]
        hs = [int(h) for h in n_harms]
        pk = torch.empty((len(hs), max(int(capacity), 1), 24), dtype=torch.uint8, device=self.device)
        nf = torch.zeros(len(hs), dtype=torch.int64, device=self.device)
        scr = torch.empty(max(self.harmonic_peaks_bytes(n, hs), 1), dtype=torch.uint8, device=self.device)
        self.harmonic_peaks_async(plane.data_ptr(), n, hs, thresholds, pk.data_ptr(), capacity, nf.data_ptr(), scr,
                                  stream)
        found, over = peak_counts(nf, len(hs), capacity, stream)
        return _capacity_result("fdas_harmonic_peaks", over, truncate,
                                [peak_records(pk[l], found[l], capacity) for l in range(len(hs))])

    def harmonic_sum_peaks(self, plane, n_harm, threshold, capacity=1 << 16, out=None, stream=None,
                           truncate=False):
        """Harmonic sum and the thresholded peaks of the summed plane in one
        call (fdas_harmonic_sum_peaks) -> (summed plane, peaks dict as from
        peaks()); overflow as for peaks()."""
        import torch
        if plane.dim() != 2 or plane.shape[0] != self.n_z or plane.dtype != self.torch_plane_dtype() \
                or not plane.is_contiguous():
            raise ValueError("plane must be a contiguous (n_z, n) tensor of the plan's plane dtype")
        n = plane.shape[1]
        nh = (n - 1) // int(n_harm) + 1 if n > 0 else 0
        if out is None:
            out = torch.empty((self.n_z, nh), dtype=plane.dtype, device=self.device)
        if out.dtype != plane.dtype or tuple(out.shape) != (self.n_z, nh) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, shape or layout")
        pk = torch.empty((max(int(capacity), 1), 24), dtype=torch.uint8, device=self.device)
        nf = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().fdas_harmonic_sum_peaks(self._h, ctypes.c_void_p(plane.data_ptr()), n, int(n_harm),
                                             ctypes.c_void_p(out.data_ptr()), float(threshold),
                                             ctypes.c_void_p(pk.data_ptr()), int(capacity),
                                             ctypes.c_void_p(nf.data_ptr()), _stream_ptr(stream)),
               "fdas_harmonic_sum_peaks")
        (found,), over = peak_counts(nf, 1, capacity, stream)
        return _capacity_result("fdas_harmonic_sum_peaks", over, truncate, (out, peak_records(pk, found, capacity)))

    def bank(self):
        """Template bank as a complex tensor view (FP32/FP64), raw bfloat16
        pairs (BF16) or e4m3 code pairs (FP8), shape (n_z, L, 2)."""
        import torch
        L = self.seg_len
        b = self.workspace[self.layout.bank_offset:self.layout.bank_offset + self.layout.bank_bytes]
        if self.cfg.compute == FP32:
            return b.view(torch.float32).view(self.n_z, L, 2)
        if self.cfg.compute == FP64:
            return b.view(torch.float64).view(self.n_z, L, 2)
        if self.cfg.compute == FP8E4M3:
            return b.view(self.n_z, L, 2)          # e4m3 codes (re, im)
        return b.view(torch.int16).view(self.n_z, L, 2)

    def fp8_exponents(self):
        """Per-template power-of-two exponents t_j of the FP8 bank (bank = e4m3(H 2^t_j))."""
        import torch
        if self.cfg.compute != FP8E4M3:
            raise ValueError("only FP8 plans have bank exponents")
        off = self.layout.tables_offset + self.n_z * self.seg_len * 8
        return self.workspace[off:off + 4 * self.n_z].view(torch.int32)


def tune(spectrum, z_min, z_step, n_z, n_taps, compute="bf16", plane_dtype=None, max_bins=None,
         seg_len=0, algo="auto", z_chunk=0, reps=5, stream=None):
    """Measured choice of seg_len / algo / z_chunk (fdas_tune) on a device
    spectrum; knobs given as non-zero are kept.  Returns a dict with the
    chosen knobs and the mean launch time in ms."""
    import torch
    n = spectrum.numel()
    cfg = make_config(max_bins or n, z_min, z_step, n_z, n_taps, seg_len, compute, plane_dtype, z_chunk, algo)
    nbytes = ctypes.c_size_t()
    _check(lib().fdas_tune_workspace(ctypes.byref(cfg), ctypes.byref(nbytes)), "fdas_tune_workspace")
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=spectrum.device)
    pdt = {FP32: torch.float32, BF16: torch.bfloat16, FP64: torch.float64}[cfg.plane_dtype]
    plane = torch.empty((int(n_z), n), dtype=pdt, device=spectrum.device)
    best = FdasConfig()
    ms = ctypes.c_float()
    _check(lib().fdas_tune(ctypes.byref(cfg), ctypes.c_void_p(spectrum.data_ptr()), n,
                           ctypes.c_void_p(plane.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes.value,
                           int(reps), ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream)), "fdas_tune")
    return {"seg_len": int(best.seg_len), "algo": {ALGO_VALU: "valu", ALGO_MFMA: "mfma"}[int(best.algo)],
            "z_chunk": int(best.z_chunk), "ms": float(ms.value)}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def prepare(series, out=None, stream=None):
    """Normalised spectrum of a real FP32 time series (fdas_prepare): the
    single-precision real FFT, Nyquist dropped, DC zeroed, median-power
    normalisation; returns an (n_t / 2,) complex64 tensor."""
    import torch
    if series.dtype != torch.float32 or series.dim() != 1 or not series.is_contiguous() or not series.is_cuda:
        raise ValueError("series must be a contiguous 1-D float32 device tensor")
    n_t = series.numel()
    nb = ctypes.c_size_t(0)
    _check(lib().fdas_prepare_workspace(n_t, ctypes.byref(nb)), "fdas_prepare_workspace")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=series.device)
    if out is None:
        out = torch.empty(n_t // 2, dtype=torch.complex64, device=series.device)
    elif out.dtype != torch.complex64 or out.numel() != n_t // 2 or not out.is_contiguous():
        raise ValueError("out must be a contiguous complex64 tensor of n_t / 2 bins")
    _check(lib().fdas_prepare(ctypes.c_void_p(series.data_ptr()), n_t, ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), nb.value, _stream_ptr(stream)), "fdas_prepare")
    return out


def refine(spectrum, r, z, taps=32, n_steps=0, eta_r_scale=1.0, eta_z_scale=1.0, stream=None):
    """fdas_refine on device tensors.  r, z: float64 start points (copied);
    returns (r, z, power, dP/dr, dP/dz) float64 tensors at the final points."""
    import torch
    if spectrum.dtype != torch.complex64 or not spectrum.is_contiguous():
        raise ValueError("spectrum must be a contiguous complex64 tensor")
    r = r.to(device=spectrum.device, dtype=torch.float64).contiguous().clone()
    z = z.to(device=spectrum.device, dtype=torch.float64).contiguous().clone()
    if r.shape != z.shape or r.dim() != 1:
        raise ValueError("r and z must be 1-D tensors of equal length")
    n = r.numel()
    P = torch.empty_like(r)
    gr = torch.empty_like(r)
    gz = torch.empty_like(r)
    _check(lib().fdas_refine(ctypes.c_void_p(spectrum.data_ptr()), spectrum.numel(), n, _ptr(r),
                             _ptr(z), _ptr(P), _ptr(gr), _ptr(gz), int(taps), int(n_steps),
                             float(eta_r_scale), float(eta_z_scale), _stream_ptr(stream)),
           "fdas_refine")
    return r, z, P, gr, gz


def _make_power_fn():
    import torch

    class InterpolatedPower(torch.autograd.Function):
        """P(r, z) of the taps-bin interpolated matched filter; the backward
        pass is the library's fdas_refine_backward kernel."""

        @staticmethod
        def forward(ctx, r, z, spectrum, taps):
            _, _, P, _, _ = refine(spectrum, r.detach(), z.detach(), taps=taps, n_steps=0)
            ctx.save_for_backward(r.detach().to(torch.float64).contiguous(),
                                  z.detach().to(torch.float64).contiguous())
            ctx.spectrum = spectrum
            ctx.taps = taps
            return P.to(r.dtype)

        @staticmethod
        def backward(ctx, grad_p):
            r, z = ctx.saved_tensors
            g = grad_p.to(torch.float64).contiguous()
            gr = torch.empty_like(r)
            gz = torch.empty_like(r)
            _check(lib().fdas_refine_backward(
                ctypes.c_void_p(ctx.spectrum.data_ptr()), ctx.spectrum.numel(), r.numel(), _ptr(r),
                _ptr(z), _ptr(g), _ptr(gr), _ptr(gz), int(ctx.taps), _stream_ptr(None)),
                "fdas_refine_backward")
            return gr.to(grad_p.dtype), gz.to(grad_p.dtype), None, None

    return InterpolatedPower


_power_fn = None


def interpolated_power(r, z, spectrum, taps=32):
    """Differentiable P(r, z) (torch.autograd) on device tensors r, z."""
    global _power_fn
    if _power_fn is None:
        _power_fn = _make_power_fn()
    return _power_fn.apply(r, z, spectrum, taps)
