"""Host-side checks of the C ABI: the library loads, exports every function
the header declares, and rejects bad arguments without touching a device."""
import ctypes

import pytest

from paper_2206_12205_amd import fdas as F


def make(**kw):
    base = dict(max_bins=65536, z_min=-16.0, z_step=2.0, n_z=17, n_taps=64, seg_len=1024,
                compute="fp32", plane_dtype=None, z_chunk=0)
    base.update(kw)
    return F.make_config(**base)


def plan_status(cfg):
    h = ctypes.c_void_p()
    n = ctypes.c_size_t()
    s = F.lib().fdas_plan(ctypes.byref(cfg), ctypes.byref(h), ctypes.byref(n))
    if s == F.OK:
        F.lib().fdas_destroy(h)
    return s, n.value


def test_library_exports_every_header_function():
    names = F.header_functions()
    assert "fdas_correlate" in names and "fdas_plan" in names and len(names) >= 10
    L = F.lib()
    for nm in names:
        assert hasattr(L, nm), nm
    assert F.lib().fdas_version().decode().count(".") == 2


def test_struct_sizes():
    assert ctypes.sizeof(F.FdasPeak) == 24
    assert ctypes.sizeof(F.FdasConfig) == 56
    assert ctypes.sizeof(F.FdasLayout) == 7 * 8 + 5 * 4 + 4 + 2 * 8


@pytest.mark.parametrize("kw,want", [
    (dict(), F.OK),
    (dict(n_taps=63), F.E_INVALID),          # odd M
    (dict(n_taps=0), F.E_INVALID),
    (dict(n_taps=1024), F.E_INVALID),        # M >= L
    (dict(seg_len=3000), F.E_INVALID),       # not a power of two
    (dict(seg_len=512), F.E_INVALID),        # below the supported range
    (dict(seg_len=32768), F.E_INVALID),
    (dict(n_z=0), F.E_INVALID),
    (dict(max_bins=0), F.E_INVALID),
    (dict(z_step=0.0), F.E_INVALID),
    (dict(n_z=1, z_step=0.0), F.OK),         # a single template needs no step
    (dict(compute="fp8"), F.OK),
    (dict(compute="fp8", seg_len=8192, n_taps=256), F.E_UNSUPPORTED),   # FP8: L <= 4096
    (dict(compute="fp8", seg_len=4096, n_taps=256, algo="mfma"), F.E_UNSUPPORTED),
    (dict(compute="fp8", plane_dtype="fp64"), F.E_INVALID),
    (dict(compute="fp8", seg_len=0, n_taps=256), F.OK),
    (dict(compute=7), F.E_INVALID),
    (dict(compute="fp64", plane_dtype="fp32"), F.E_INVALID),
    (dict(compute="fp32", plane_dtype="fp64"), F.E_INVALID),
    (dict(compute="fp64", seg_len=16384, n_taps=512), F.E_UNSUPPORTED),
    (dict(compute="bf16", plane_dtype="fp32"), F.OK),
    (dict(z_chunk=-1), F.E_INVALID),
    (dict(seg_len=0, n_taps=256), F.OK),     # automatic L
    (dict(compute="bf16", seg_len=8192, n_taps=256, algo="mfma"), F.OK),
    (dict(compute="fp32", seg_len=8192, n_taps=256, algo="mfma"), F.E_UNSUPPORTED),
    (dict(compute="bf16", seg_len=4096, n_taps=256, algo="mfma"), F.OK),
    (dict(compute="bf16", seg_len=2048, n_taps=256, algo="mfma"), F.E_UNSUPPORTED),
    (dict(algo=3), F.E_INVALID),
])
def test_plan_validation(kw, want):
    assert plan_status(make(**kw))[0] == want


def test_layout_and_workspace_checks_on_host():
    L = F.lib()
    cfg = make(max_bins=4096, seg_len=0, n_taps=256, n_z=5, z_min=-4.0, compute="bf16")
    h = ctypes.c_void_p()
    n = ctypes.c_size_t()
    assert L.fdas_plan(ctypes.byref(cfg), ctypes.byref(h), ctypes.byref(n)) == F.OK
    try:
        lay = F.FdasLayout()
        assert L.fdas_get_layout(h, ctypes.byref(lay)) == F.OK
        assert lay.seg_len == 4096 and lay.valid_per_seg == 4096 - 256
        assert lay.bank_bytes == 5 * 4096 * 4 and lay.total_bytes == n.value
        assert lay.algo == F.ALGO_MFMA and lay.tables_bytes > 0
        assert lay.tables_offset + lay.tables_bytes <= lay.total_bytes
        assert lay.bank_offset % 256 == 0 and lay.twiddle_offset % 256 == 0
        fake = ctypes.c_void_p(0x10000)           # never dereferenced on these paths
        assert L.fdas_correlate(h, fake, 100, fake, None) == F.E_WORKSPACE
        assert L.fdas_make_templates_jerk(h, 12.0, None) == F.E_WORKSPACE
        assert L.fdas_make_templates_jerk(h, float("nan"), None) == F.E_INVALID
        assert L.fdas_make_templates_jerk(None, 12.0, None) == F.E_INVALID
        assert L.fdas_set_workspace(h, fake, n.value - 1) == F.E_WORKSPACE
        assert L.fdas_set_workspace(h, ctypes.c_void_p(0x10008), n.value) == F.E_INVALID
        assert L.fdas_set_workspace(h, None, n.value) == F.E_WORKSPACE
        assert L.fdas_set_workspace(h, fake, n.value) == F.OK
        assert L.fdas_correlate(h, fake, 100, fake, None) == F.E_STATE      # no templates yet
        assert L.fdas_correlate(h, fake, 0, fake, None) == F.E_INVALID
        assert L.fdas_correlate(h, fake, 4097, fake, None) == F.E_INVALID
        assert L.fdas_correlate(h, ctypes.c_void_p(0x10004), 100, fake, None) == F.E_INVALID
        assert L.fdas_correlate(h, None, 100, fake, None) == F.E_INVALID
        nf = ctypes.c_void_p(0x20000)
        assert L.fdas_peaks(h, fake, 100, 1.0, None, 5, nf, None) == F.E_INVALID   # capacity>0, no out
        assert L.fdas_peaks(h, fake, 100, 1.0, fake, -1, nf, None) == F.E_INVALID
        assert L.fdas_peaks(h, fake, 100, 1.0, fake, 5, ctypes.c_void_p(0x20004), None) == F.E_INVALID
        # band maxima: argument checks only
        assert L.fdas_band_max(h, fake, 100, fake, 0, fake, None) == F.E_INVALID
        assert L.fdas_band_max(h, fake, 100, fake, 65536, fake, None) == F.E_INVALID
        assert L.fdas_band_max(h, fake, 0, fake, 4, fake, None) == F.E_INVALID
        assert L.fdas_band_max(h, fake, 100, ctypes.c_void_p(0x10004), 4, fake, None) == F.E_INVALID
        assert L.fdas_band_max(h, fake, 100, fake, 4, ctypes.c_void_p(0x10008), None) == F.E_INVALID
        assert L.fdas_band_max(h, fake, 100, None, 4, fake, None) == F.E_INVALID
        # harmonic sum: argument checks only (each returns before any launch)
        assert L.fdas_harmonic_sum(h, fake, 100, 0, fake, None) == F.E_INVALID
        assert L.fdas_harmonic_sum(h, fake, 100, 33, fake, None) == F.E_INVALID
        assert L.fdas_harmonic_sum(h, fake, 0, 4, fake, None) == F.E_INVALID
        assert L.fdas_harmonic_sum(h, fake, 4097, 4, fake, None) == F.E_INVALID
        assert L.fdas_harmonic_sum(h, None, 100, 4, fake, None) == F.E_INVALID
        assert L.fdas_harmonic_sum(h, fake, 100, 4, None, None) == F.E_INVALID
        assert L.fdas_harmonic_sum(h, ctypes.c_void_p(0x10001), 100, 4, fake, None) == F.E_INVALID
        assert L.fdas_harmonic_sum(None, fake, 100, 4, fake, None) == F.E_INVALID
        # several harmonic sums: argument checks only
        H3 = (ctypes.c_int32 * 3)(2, 4, 8)
        Hbad = (ctypes.c_int32 * 3)(2, 2, 8)
        Hbig = (ctypes.c_int32 * 1)(33)
        O3 = (ctypes.c_void_p * 3)(0x10000, 0x20000, 0x30000)
        O3bad = (ctypes.c_void_p * 3)(0x10000, None, 0x30000)
        assert L.fdas_harmonic_sums(h, fake, 100, 3, Hbad, O3, None) == F.E_INVALID     # not increasing
        assert L.fdas_harmonic_sums(h, fake, 100, 1, Hbig, O3, None) == F.E_INVALID     # H > 32
        assert L.fdas_harmonic_sums(h, fake, 100, 3, H3, O3bad, None) == F.E_INVALID    # missing output
        assert L.fdas_harmonic_sums(h, fake, 100, 0, H3, O3, None) == F.E_INVALID
        assert L.fdas_harmonic_sums(h, fake, 100, 9, H3, O3, None) == F.E_INVALID
        assert L.fdas_harmonic_sums(h, fake, 4097, 3, H3, O3, None) == F.E_INVALID
        assert L.fdas_harmonic_sums(h, None, 100, 3, H3, O3, None) == F.E_INVALID
        sb = ctypes.c_size_t(0)
        assert L.fdas_harmonic_sums_peaks_workspace(h, 100, 3, H3, ctypes.byref(sb)) == F.OK and sb.value > 0
        assert L.fdas_harmonic_sums_peaks_workspace(h, 100, 3, Hbad, ctypes.byref(sb)) == F.E_INVALID
        T3 = (ctypes.c_float * 3)(1.0, 2.0, 3.0)
        assert L.fdas_harmonic_sums_peaks(h, fake, 100, 3, H3, O3, T3, O3, 5, nf, fake, 1, None) == F.E_WORKSPACE
        assert L.fdas_harmonic_sums_peaks(h, fake, 100, 3, H3, O3, None, O3, 5, nf, fake, 1 << 20, None) \
            == F.E_INVALID
        # harmonic sum with peaks: argument checks only
        assert L.fdas_harmonic_sum_peaks(h, fake, 100, 0, fake, 1.0, fake, 5, nf, None) == F.E_INVALID
        assert L.fdas_harmonic_sum_peaks(h, fake, 100, 33, fake, 1.0, fake, 5, nf, None) == F.E_INVALID
        assert L.fdas_harmonic_sum_peaks(h, fake, 4097, 4, fake, 1.0, fake, 5, nf, None) == F.E_INVALID
        assert L.fdas_harmonic_sum_peaks(h, fake, 100, 4, fake, 1.0, None, 5, nf, None) == F.E_INVALID
        assert L.fdas_harmonic_sum_peaks(h, fake, 100, 4, fake, 1.0, fake, -1, nf, None) == F.E_INVALID
        assert L.fdas_harmonic_sum_peaks(h, fake, 100, 4, fake, 1.0, ctypes.c_void_p(0x10008), 5, nf, None) \
            == F.E_INVALID
        assert L.fdas_harmonic_sum_peaks(h, fake, 100, 4, None, 1.0, fake, 5, nf, None) == F.E_INVALID
        assert L.fdas_harmonic_sum_peaks(None, fake, 100, 4, fake, 1.0, fake, 5, nf, None) == F.E_INVALID
        # fused plane + peaks: argument and state checks only (no launch)
        assert L.fdas_correlate_peaks(h, fake, 100, fake, 1.0, fake, 5, nf, None) == F.E_STATE   # no templates
        assert L.fdas_correlate_peaks(h, fake, 100, fake, 1.0, None, 5, nf, None) == F.E_INVALID
        assert L.fdas_correlate_peaks(h, fake, 100, fake, 1.0, fake, -1, nf, None) == F.E_INVALID
        assert L.fdas_correlate_peaks(h, fake, 100, fake, 1.0, fake, 5, ctypes.c_void_p(0x20004), None) \
            == F.E_INVALID
        assert L.fdas_correlate_peaks(h, fake, 0, fake, 1.0, fake, 5, nf, None) == F.E_INVALID
        assert L.fdas_correlate_peaks(h, fake, 4097, fake, 1.0, fake, 5, nf, None) == F.E_INVALID
        assert L.fdas_correlate_peaks(h, ctypes.c_void_p(0x10008), 100, fake, 1.0, fake, 5, nf, None) \
            == F.E_INVALID
        assert L.fdas_correlate_peaks(None, fake, 100, fake, 1.0, fake, 5, nf, None) == F.E_INVALID
        sb = ctypes.c_size_t(0)
        assert L.fdas_batch_peaks_workspace(h, ctypes.byref(sb)) == F.E_STATE               # no batch
        assert L.fdas_batch_peaks_workspace(h, None) == F.E_INVALID
        assert L.fdas_correlate_batch_peaks(h, fake, fake, 1.0, fake, 5, nf, fake, 1 << 20, None) == F.E_STATE
        assert L.fdas_correlate_batch_peaks(h, fake, fake, 1.0, None, 5, nf, fake, 1 << 20, None) == F.E_INVALID
        assert L.fdas_correlate_batch_peaks(h, fake, fake, 1.0, fake, 5, None, fake, 1 << 20, None) \
            == F.E_INVALID
    finally:
        L.fdas_destroy(h)
    L.fdas_destroy(None)
    assert L.fdas_strerror(F.E_CAPACITY).decode() == "peak capacity exceeded"


def test_prepare_argument_checks():
    L = F.lib()
    nb = ctypes.c_size_t(0)
    assert L.fdas_prepare_workspace(1 << 20, ctypes.byref(nb)) == F.OK
    assert nb.value >= (1 << 19) * 16
    # 3 * 2^a lengths: the four-step form, 3 * 2^7 .. 3 * 2^22 samples
    for n_t in (3 << 7, 3 << 10, 3 << 22):
        assert L.fdas_prepare_workspace(n_t, ctypes.byref(nb)) == F.OK, n_t
        assert nb.value >= (n_t // 2) * 16
    for n_t in (3 << 6, 3 << 23, 5 << 10, 6, 1000):
        assert L.fdas_prepare_workspace(n_t, ctypes.byref(nb)) == F.E_UNSUPPORTED, n_t
    assert L.fdas_prepare_workspace(2, ctypes.byref(nb)) == F.E_INVALID
    assert L.fdas_prepare_workspace(1024, None) == F.E_INVALID
    fake = ctypes.c_void_p(0x10000)
    assert L.fdas_prepare(None, 1024, fake, fake, 1 << 20, None) == F.E_INVALID
    assert L.fdas_prepare(ctypes.c_void_p(0x10004), 1024, fake, fake, 1 << 20, None) == F.E_INVALID
    assert L.fdas_prepare(fake, 1024, ctypes.c_void_p(0x10008), fake, 1 << 20, None) == F.E_INVALID
    assert L.fdas_prepare(fake, 1000, fake, fake, 1 << 20, None) == F.E_UNSUPPORTED
    assert L.fdas_prepare(fake, 1024, fake, fake, 16, None) == F.E_WORKSPACE
    assert L.fdas_prepare(fake, 1024, fake, None, 1 << 20, None) == F.E_WORKSPACE


def test_peaks_check_argument_checks_on_host():
    """fdas_peaks_check (the synchronous overflow check): bad arguments are
    refused before any device call."""
    import ctypes
    L = F.lib()
    counts = (ctypes.c_int64 * 4)()
    fake = ctypes.c_void_p(0x10000)
    assert L.fdas_peaks_check(None, 1, 5, counts, None) == F.E_INVALID
    assert L.fdas_peaks_check(fake, 1, 5, None, None) == F.E_INVALID
    assert L.fdas_peaks_check(fake, 0, 5, counts, None) == F.E_INVALID
    assert L.fdas_peaks_check(fake, 1, -1, counts, None) == F.E_INVALID
    assert L.fdas_peaks_check(ctypes.c_void_p(0x10004), 1, 5, counts, None) == F.E_INVALID


def test_null_arguments():
    L = F.lib()
    assert L.fdas_plan(None, None, None) == F.E_INVALID
    assert L.fdas_make_templates(None, None) == F.E_INVALID
    assert L.fdas_get_layout(None, None) == F.E_INVALID


def test_refine_argument_checks_on_host():
    L = F.lib()
    fake = ctypes.c_void_p(0x10000)
    D = ctypes.c_double
    args = lambda **kw: [kw.get("spec", fake), kw.get("n", 100), kw.get("nc", 4), fake, fake, fake, fake, fake,
                         kw.get("taps", 32), kw.get("steps", 0), D(1.0), D(kw.get("eta", 1.0)), None]
    assert L.fdas_refine(*args(taps=31)) == F.E_INVALID
    assert L.fdas_refine(*args(taps=66)) == F.E_INVALID
    assert L.fdas_refine(*args(taps=0)) == F.E_INVALID
    assert L.fdas_refine(*args(nc=-1)) == F.E_INVALID
    assert L.fdas_refine(*args(steps=-1)) == F.E_INVALID
    assert L.fdas_refine(*args(n=0)) == F.E_INVALID
    assert L.fdas_refine(*args(spec=ctypes.c_void_p(0x10004))) == F.E_INVALID
    assert L.fdas_refine(*args(spec=None)) == F.E_INVALID
    assert L.fdas_refine(*args(eta=float("nan"))) == F.E_INVALID
    assert L.fdas_refine_backward(fake, 100, 4, fake, fake, fake, fake, fake, 33, None) == F.E_INVALID
    assert L.fdas_refine_backward(fake, 100, 4, fake, None, fake, fake, fake, 32, None) == F.E_INVALID


def test_batch_argument_checks_on_host():
    L = F.lib()
    cfg = make(max_bins=4096, seg_len=0, n_taps=256, n_z=5, z_min=-4.0, compute="bf16", max_jobs=3)
    assert plan_status(make(max_jobs=-1))[0] == F.E_INVALID
    assert ctypes.sizeof(F.FdasJob) == 24
    h = ctypes.c_void_p()
    n = ctypes.c_size_t()
    assert L.fdas_plan(ctypes.byref(cfg), ctypes.byref(h), ctypes.byref(n)) == F.OK
    try:
        fake = ctypes.c_void_p(0x10000)           # never dereferenced on these paths
        jobs = (F.FdasJob * 4)(F.FdasJob(0, 100, 0), F.FdasJob(100, 50, 500), F.FdasJob(150, 4096, 750),
                               F.FdasJob(0, 1, 0))
        assert L.fdas_set_batch(h, jobs, 2, 1000, 10 ** 6, None) == F.E_WORKSPACE
        assert L.fdas_set_workspace(h, fake, n.value) == F.OK
        big = 10 ** 6
        assert L.fdas_set_batch(h, jobs, 0, big, big, None) == F.E_INVALID
        assert L.fdas_set_batch(h, None, 1, big, big, None) == F.E_INVALID
        assert L.fdas_set_batch(h, jobs, 4, big, big * 10, None) == F.E_INVALID     # above max_jobs
        assert L.fdas_set_batch(h, jobs, 3, 4245, big, None) == F.E_INVALID        # spectra too short
        assert L.fdas_set_batch(h, jobs, 3, 4246, 750 + 5 * 4096 - 1, None) == F.E_INVALID  # planes too short
        bad = (F.FdasJob * 1)(F.FdasJob(0, 4097, 0))                                # above max_bins
        assert L.fdas_set_batch(h, bad, 1, big, big * 10, None) == F.E_INVALID
        bad = (F.FdasJob * 1)(F.FdasJob(0, 0, 0))                                   # empty spectrum
        assert L.fdas_set_batch(h, bad, 1, big, big, None) == F.E_INVALID
        bad = (F.FdasJob * 1)(F.FdasJob(-1, 10, 0))
        assert L.fdas_set_batch(h, bad, 1, big, big, None) == F.E_INVALID
        bad = (F.FdasJob * 1)(F.FdasJob(0, 10, -5))
        assert L.fdas_set_batch(h, bad, 1, big, big, None) == F.E_INVALID
        assert L.fdas_correlate_batch(h, fake, fake, None) == F.E_STATE            # no templates, no batch
        assert L.fdas_correlate_batch(h, ctypes.c_void_p(0x10008), fake, None) == F.E_INVALID
        assert L.fdas_correlate_batch(h, None, fake, None) == F.E_INVALID
    finally:
        L.fdas_destroy(h)
    cfg0 = make(max_bins=4096, n_z=5, z_min=-4.0)     # max_jobs = 0: no batches
    assert L.fdas_plan(ctypes.byref(cfg0), ctypes.byref(h), ctypes.byref(n)) == F.OK
    try:
        assert L.fdas_set_workspace(h, ctypes.c_void_p(0x10000), n.value) == F.OK
        jobs = (F.FdasJob * 1)(F.FdasJob(0, 100, 0))
        assert L.fdas_set_batch(h, jobs, 1, 100, 500, None) == F.E_INVALID
    finally:
        L.fdas_destroy(h)


def test_tune_argument_checks_on_host():
    L = F.lib()
    cfg = make(max_bins=4096, seg_len=0, n_taps=256, n_z=5, z_min=-4.0, compute="bf16")
    n = ctypes.c_size_t()
    assert L.fdas_tune_workspace(ctypes.byref(cfg), ctypes.byref(n)) == F.OK
    # covers the largest candidate: L = 16384 on the vector-ALU kernel
    big = make(max_bins=4096, seg_len=16384, n_taps=256, n_z=5, z_min=-4.0, compute="bf16", algo="valu")
    assert n.value >= plan_status(big)[1] > 0
    need = n.value
    fixed = ctypes.c_size_t()
    c4 = make(max_bins=4096, seg_len=4096, n_taps=256, n_z=5, z_min=-4.0, compute="bf16", algo="mfma", z_chunk=5)
    assert L.fdas_tune_workspace(ctypes.byref(c4), ctypes.byref(fixed)) == F.OK
    assert fixed.value == plan_status(c4)[1]
    bad = make(n_z=0)
    assert L.fdas_tune_workspace(ctypes.byref(bad), ctypes.byref(n)) == F.E_INVALID
    assert L.fdas_tune_workspace(None, ctypes.byref(n)) == F.E_INVALID
    c64 = make(compute="fp64", seg_len=16384, n_taps=512)
    assert L.fdas_tune_workspace(ctypes.byref(c64), ctypes.byref(n)) == F.E_UNSUPPORTED
    fake = ctypes.c_void_p(0x10000)
    best = F.FdasConfig()
    ms = ctypes.c_float()
    args = lambda **kw: [ctypes.byref(kw.get("cfg", cfg)), fake, kw.get("nb", 100), fake, fake,
                         kw.get("ws", 1 << 40), kw.get("reps", 3), ctypes.byref(best), ctypes.byref(ms), None]
    assert L.fdas_tune(*args(reps=0)) == F.E_INVALID
    assert L.fdas_tune(*args(reps=1001)) == F.E_INVALID
    assert L.fdas_tune(*args(nb=0)) == F.E_INVALID
    assert L.fdas_tune(*args(nb=4097)) == F.E_INVALID
    assert L.fdas_tune(*args(ws=need - 1)) == F.E_WORKSPACE


def test_fp8_layout_on_host():
    L = F.lib()
    cfg = make(max_bins=100000, seg_len=0, n_taps=256, n_z=9, z_min=-8.0, compute="fp8")
    h = ctypes.c_void_p()
    n = ctypes.c_size_t()
    assert L.fdas_plan(ctypes.byref(cfg), ctypes.byref(h), ctypes.byref(n)) == F.OK
    try:
        lay = F.FdasLayout()
        assert L.fdas_get_layout(h, ctypes.byref(lay)) == F.OK
        assert lay.seg_len == 4096 and lay.algo == F.ALGO_VALU and lay.bank_elem_bytes == 2
        assert lay.bank_bytes == 9 * 4096 * 2
        assert lay.tables_bytes == 9 * 4096 * 8 + 9 * 4      # FP32 staging + exponents
    finally:
        L.fdas_destroy(h)


def test_sums_peaks_noalloc_checks_on_host():
    """fdas_harmonic_sums_peaks_noalloc: bad arguments and a scratch need above
    FDAS_NOALLOC_SCRATCH_BYTES are refused before any device call."""
    L = F.lib()
    P = ctypes.c_void_p

    def call(h, n, hs, plane=0x10000, n_found=0x20000, cap=16):
        k = len(hs)
        harr = (ctypes.c_int32 * k)(*hs)
        outs = (P * k)(*[0x30000 + 0x1000 * i for i in range(k)])
        thr = (ctypes.c_float * k)(*[10.0] * k)
        pks = (P * k)(*[0x40000 + 0x1000 * i for i in range(k)])
        return L.fdas_harmonic_sums_peaks_noalloc(h, P(plane), n, k, harr, outs, thr, pks, cap, P(n_found), None)

    def with_plan(cfg, fn):
        h = P()
        nb = ctypes.c_size_t()
        assert L.fdas_plan(ctypes.byref(cfg), ctypes.byref(h), ctypes.byref(nb)) == F.OK
        try:
            return fn(h)
        finally:
            L.fdas_destroy(h)

    assert call(None, 1000, [2, 4]) == F.E_INVALID
    small = make(compute="bf16", plane_dtype="bf16")
    assert with_plan(small, lambda h: call(h, 1000, [2, 4], plane=0)) == F.E_INVALID
    assert with_plan(small, lambda h: call(h, 1000, [2, 4], n_found=0x20004)) == F.E_INVALID   # 8-byte aligned
    assert with_plan(small, lambda h: call(h, 1000, [4, 2])) == F.E_INVALID                    # increasing H
    assert with_plan(small, lambda h: call(h, 0, [2])) == F.E_INVALID
    assert with_plan(small, lambda h: call(h, 65537, [2])) == F.E_INVALID                      # > max_bins

    # a plane whose scratch need exceeds the fixed array: FDAS_E_WORKSPACE
    # (computed from the workspace query, no device touched)
    big = make(max_bins=1 << 24, n_z=801, z_min=-800.0, compute="bf16", plane_dtype="bf16")

    def too_big(h):
        hs = [2, 4, 8, 16]
        need = ctypes.c_size_t()
        assert L.fdas_harmonic_sums_peaks_workspace(h, 1 << 24, 4, (ctypes.c_int32 * 4)(*hs),
                                                    ctypes.byref(need)) == F.OK
        assert need.value > F.NOALLOC_SCRATCH_BYTES
        return call(h, 1 << 24, hs)
    assert with_plan(big, too_big) == F.E_WORKSPACE


def test_batch_sums_checks_on_host():
    """fdas_batch_harmonic_sums_peaks(_workspace): bad levels are refused and
    a plan with no stored batch answers FDAS_E_STATE, before any device call."""
    L = F.lib()
    P = ctypes.c_void_p
    h = P()
    nb = ctypes.c_size_t()
    assert L.fdas_plan(ctypes.byref(make(compute="bf16", plane_dtype="bf16")), ctypes.byref(h),
                       ctypes.byref(nb)) == F.OK
    try:
        def ws(hs):
            need = ctypes.c_size_t()
            return L.fdas_batch_harmonic_sums_peaks_workspace(h, len(hs), (ctypes.c_int32 * len(hs))(*hs),
                                                              ctypes.byref(need))

        def run(hs):
            k = len(hs)
            return L.fdas_batch_harmonic_sums_peaks(h, P(0x10000), k, (ctypes.c_int32 * k)(*hs),
                                                    (ctypes.c_float * k)(*[10.0] * k), P(0x40000), 16,
                                                    P(0x20000), P(0x50000), 1 << 20, None)
        assert ws([]) == F.E_INVALID
        assert ws([4, 2]) == F.E_INVALID                  # increasing H
        assert ws(list(range(2, 11))) == F.E_INVALID      # more than 8 levels
        assert ws([2, 4]) == F.E_STATE                    # no batch stored
        assert run([2, 4]) == F.E_STATE
        assert L.fdas_batch_harmonic_sums_peaks_workspace(h, 2, (ctypes.c_int32 * 2)(2, 4), None) == F.E_INVALID
    finally:
        L.fdas_destroy(h)


def test_harmonic_sums_refuse_rows_of_4_gb():
    """The summing kernels address a row with 32-bit offsets: a plan whose
    rows would reach 4 GB less 1 MB gets FDAS_E_UNSUPPORTED from every
    harmonic-sum call (checked on the host, no device touched)."""
    L = F.lib()
    P = ctypes.c_void_p
    big = 1 << 31          # bins: 4 GB of BF16 values per row
    h = P()
    nb = ctypes.c_size_t()
    assert L.fdas_plan(ctypes.byref(make(max_bins=big, n_z=3, z_min=-2.0, compute="bf16", plane_dtype="bf16")),
                       ctypes.byref(h), ctypes.byref(nb)) == F.OK
    try:
        hs = (ctypes.c_int32 * 2)(2, 4)
        outs = (P * 2)(P(0x30000), P(0x40000))
        assert L.fdas_harmonic_sum(h, P(0x10000), big, 2, P(0x20000), None) == F.E_UNSUPPORTED
        assert L.fdas_harmonic_sums(h, P(0x10000), big, 2, hs, outs, None) == F.E_UNSUPPORTED
        need = ctypes.c_size_t()
        assert L.fdas_harmonic_sums_peaks_workspace(h, big, 2, hs, ctypes.byref(need)) == F.E_UNSUPPORTED
        assert L.fdas_harmonic_peaks_workspace(h, big, 2, hs, ctypes.byref(need)) == F.E_UNSUPPORTED
        # a row just below the limit is accepted by the host checks
        ok = (0xfff00000 // 2) - 1
        assert L.fdas_harmonic_sums_peaks_workspace(h, ok, 2, hs, ctypes.byref(need)) == F.OK
        assert L.fdas_harmonic_peaks_workspace(h, ok, 2, hs, ctypes.byref(need)) == F.OK
    finally:
        L.fdas_destroy(h)


def test_harmonic_peaks_checks_on_host():
    """fdas_harmonic_peaks(_workspace): the scratch size follows the plane
    length and levels, bad lists, lengths and pointers are refused and a
    short scratch answers FDAS_E_WORKSPACE, all before any device call; a plan
    with no workspace or batch is enough."""
    L = F.lib()
    P = ctypes.c_void_p
    h = P()
    nb = ctypes.c_size_t()
    assert L.fdas_plan(ctypes.byref(make(compute="bf16", plane_dtype="bf16")), ctypes.byref(h),
                       ctypes.byref(nb)) == F.OK
    try:
        def ws(n, hs):
            need = ctypes.c_size_t()
            s = L.fdas_harmonic_peaks_workspace(h, n, len(hs), (ctypes.c_int32 * len(hs))(*hs), ctypes.byref(need))
            return s, need.value

        def run(n, hs, plane=P(0x10000), peaks=P(0x40000), cap=16, n_found=P(0x20000), scratch=P(0x50000),
                nbytes=1 << 30, thr=True):
            k = len(hs)
            t = (ctypes.c_float * k)(*[10.0] * k) if thr else None
            return L.fdas_harmonic_peaks(h, plane, n, k, (ctypes.c_int32 * k)(*hs), t, peaks, cap, n_found,
                                         scratch, nbytes, None)
        s1, b1 = ws(4096, [2, 4])
        s2, b2 = ws(65536, [2, 4])
        s3, b3 = ws(65536, [2, 4, 8, 16])
        assert s1 == s2 == s3 == F.OK and 0 < b1 < b2 < b3
        assert ws(0, [2])[0] == F.E_INVALID                  # empty plane
        assert ws(65537, [2])[0] == F.E_INVALID              # above max_bins
        assert ws(4096, [])[0] == F.E_INVALID
        assert ws(4096, [4, 2])[0] == F.E_INVALID            # increasing H
        assert ws(4096, [33])[0] == F.E_INVALID              # at most 32 harmonics
        assert ws(4096, list(range(2, 11)))[0] == F.E_INVALID   # at most 8 levels
        assert L.fdas_harmonic_peaks_workspace(h, 4096, 1, (ctypes.c_int32 * 1)(2), None) == F.E_INVALID
        assert run(4096, [2], plane=None) == F.E_INVALID
        assert run(4096, [2], thr=False) == F.E_INVALID
        assert run(4096, [2], n_found=None) == F.E_INVALID
        assert run(4096, [2], n_found=P(0x20004)) == F.E_INVALID     # n_found 8-byte aligned
        assert run(4096, [2], peaks=None) == F.E_INVALID             # capacity > 0 needs peaks
        assert run(4096, [2], peaks=P(0x40008)) == F.E_INVALID       # peaks 16-byte aligned
        assert run(4096, [2], plane=P(0x10001)) == F.E_INVALID       # bfloat16 alignment
        assert run(4096, [2], cap=-1) == F.E_INVALID
        assert run(4096, [2], scratch=None) == F.E_WORKSPACE
        assert run(4096, [2], scratch=P(0x50008)) == F.E_WORKSPACE   # scratch 16-byte aligned
        assert run(4096, [2, 4], nbytes=b1 - 1) == F.E_WORKSPACE
        assert L.fdas_harmonic_peaks(None, P(0x10000), 4096, 1, (ctypes.c_int32 * 1)(2), (ctypes.c_float * 1)(1.0),
                                     P(0x40000), 4, P(0x20000), P(0x50000), 1 << 30, None) == F.E_INVALID
    finally:
        L.fdas_destroy(h)
