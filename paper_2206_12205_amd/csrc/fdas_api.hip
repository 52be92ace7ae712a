// C ABI of libfdas: plan validation, workspace layout and dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.hpp"
#include "marks.hpp"
#include "mfma4096.hpp"
#include "mfma8192.hpp"

namespace {
thread_local int g_last_hip = 0;
}  // namespace

namespace fdas {
int hip_status_of(hipError_t e) {
    if (e == hipSuccess) return FDAS_OK;
    g_last_hip = (int)e;
    return FDAS_E_HIP;
}
}  // namespace fdas

namespace {

int hip_status(hipError_t e) { return fdas::hip_status_of(e); }

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
static bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

int elem_bytes(int dtype) {
    switch (dtype) {
        case FDAS_FP32: return 8;
        case FDAS_BF16: return 4;
        case FDAS_FP64: return 16;
        case FDAS_FP8E4M3: return 2;
        default: return 0;
    }
}

// Scratch of fdas_harmonic_sums_peaks_noalloc: one fixed array per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel (in host code it is a host-side stand-in): the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoallocScratchBytes = FDAS_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
hipError_t noalloc_scratch(unsigned char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char *fdas_version(void) { return "0.1.0"; }

const char *fdas_strerror(int s) {
    switch (s) {
        case FDAS_OK: return "ok";
        case FDAS_E_INVALID: return "invalid argument or configuration";
        case FDAS_E_WORKSPACE: return "workspace missing or too small";
        case FDAS_E_HIP: return "HIP runtime error";
        case FDAS_E_CAPACITY: return "peak capacity exceeded";
        case FDAS_E_UNSUPPORTED: return "unsupported configuration";
        case FDAS_E_STATE: return "call out of order";
        default: return "unknown status";
    }
}

int fdas_last_hip_error(void) { return g_last_hip; }

int fdas_peaks_check(const int64_t *n_found, int32_t n_lists, int64_t capacity, int64_t *counts, void *stream) {
    if (!n_found || !counts || n_lists < 1 || capacity < 0 || !aligned8(n_found)) return FDAS_E_INVALID;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(counts, n_found, sizeof(int64_t) * (size_t)n_lists, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e);
    for (int32_t i = 0; i < n_lists; ++i)
        if (counts[i] > capacity) return FDAS_E_CAPACITY;
    return FDAS_OK;
}

int fdas_plan(const fdas_config *cfg, fdas_plan_t *out, size_t *workspace_bytes) {
    if (!cfg || !out || !workspace_bytes) return FDAS_E_INVALID;
    *out = nullptr;
    const fdas_config c = *cfg;
    if (c.compute != FDAS_FP32 && c.compute != FDAS_BF16 && c.compute != FDAS_FP64 && c.compute != FDAS_FP8E4M3)
        return FDAS_E_INVALID;
    if (c.n_z < 1 || c.max_bins < 1 || c.n_taps < 2 || (c.n_taps & 1) || c.n_taps > 4096) return FDAS_E_INVALID;
    if (!std::isfinite(c.z_min) || !std::isfinite(c.z_step)) return FDAS_E_INVALID;
    if (c.n_z > 1 && !(c.z_step > 0.0)) return FDAS_E_INVALID;
    if (c.z_chunk < 0) return FDAS_E_INVALID;
    if (c.algo < FDAS_ALGO_AUTO || c.algo > FDAS_ALGO_MFMA) return FDAS_E_INVALID;
    if (c.max_jobs < 0 || c.max_jobs > (1 << 24)) return FDAS_E_INVALID;
    // plane dtype: FP64 compute writes FP64 only; FP32/BF16/FP8 compute write FP32 or BF16
    if (c.compute == FDAS_FP64) {
        if (c.plane_dtype != FDAS_FP64) return FDAS_E_INVALID;
    } else if (c.plane_dtype != FDAS_FP32 && c.plane_dtype != FDAS_BF16) {
        return FDAS_E_INVALID;
    }
    int64_t L = c.seg_len;
    if (L == 0) {
        if (c.compute == FDAS_BF16 && c.algo != FDAS_ALGO_VALU && c.n_taps <= 512) {
            L = 4096;   // the 16x16x16 matrix-core kernel; overlap waste M / L <= 12.5 %
        } else if (c.compute == FDAS_BF16 && c.algo != FDAS_ALGO_VALU && c.n_taps <= 2048) {
            L = 8192;
        } else if (c.compute == FDAS_FP8E4M3) {
            L = 4096;   // the longest FP8 segment (three scaled stages)
        } else {
            // vector-ALU kernel: the shortest power of two >= 8 M (overlap
            // waste M / L <= 12.5 %); longer segments only add a pass
            // (measured: FP32, M = 256: L = 2048 / 4096 / 8192 / 16384 ->
            // 0.74 / 0.77 / 1.20 / 3.0 ms per single-DM plane)
            L = int64_t(1) << ilog2(8 * (int64_t)c.n_taps);
            if (L < 1024) L = 1024;
            const int64_t lmax = c.compute == FDAS_FP64 ? 8192 : 16384;
            if (L > lmax) L = lmax;
        }
    }
    if (L < 1024 || L > 16384 || (L & (L - 1))) return FDAS_E_INVALID;
    if (c.n_taps >= L) return FDAS_E_INVALID;
    if (c.compute == FDAS_FP64 && L > 8192) return FDAS_E_UNSUPPORTED;
    // FP8: vector-ALU kernel only, at most three radix-16 stages
    if (c.compute == FDAS_FP8E4M3 && (L > 4096 || c.algo == FDAS_ALGO_MFMA)) return FDAS_E_UNSUPPORTED;

    fdas_plan_s *p = new (std::nothrow) fdas_plan_s();
    if (!p) return FDAS_E_INVALID;
    p->cfg = c;
    p->L = (int32_t)L;
    p->log2L = ilog2(L);
    p->cfg.seg_len = p->L;
    p->M = c.n_taps;
    p->V = p->L - p->M;
    const bool mfma_ok = c.compute == FDAS_BF16 && (L == fdas::m8k::kL || L == fdas::m4k::kL);
    if (c.algo == FDAS_ALGO_MFMA && !mfma_ok) {
        delete p;
        return FDAS_E_UNSUPPORTED;
    }
    p->mfma = mfma_ok && c.algo != FDAS_ALGO_VALU;
    int zc = c.z_chunk;
    if (zc == 0) {
        // vector-ALU and L = 8192 matrix-core kernels: eight chunks, one per
        // XCD (L = 8192, single-DM plane: 0.73 ms against 0.80 ms with four
        // chunks and 0.84-1.0 ms with 7 to 15 templates per chunk, when the
        // chunks no longer map one to an XCD).  L = 4096 matrix-core kernel: each chunk
        // repeats the segment's forward transform, so two chunks, or more
        // when the segments of max_bins give fewer than 512 workgroups (one
        // per slot of a 256-CU device at two per CU); measured on the
        // single-DM and wide planes: two chunks 1.5 % / 2 % faster than
        // three, one chunk slower.
        if (!p->mfma || L == fdas::m8k::kL) {
            zc = (c.n_z + 7) / 8;
        } else if (L == fdas::m4k::kL) {
            const int64_t segs = (c.max_bins + (L - c.n_taps) - 1) / (L - c.n_taps);
            const int64_t nc = std::max<int64_t>(2, (512 + segs - 1) / segs);
            zc = (int)((c.n_z + nc - 1) / nc);
        }
    }
    if (zc > c.n_z) zc = c.n_z;
    p->z_chunk = zc;
    p->n_chunks = (c.n_z + zc - 1) / zc;
    p->cfg.z_chunk = zc;
    p->bank_elem = elem_bytes(c.compute);
    p->tw_elem = c.compute == FDAS_FP64 ? 16 : 8;

    size_t off = 0;
    p->off_bank = off;
    p->sz_bank = (size_t)c.n_z * (size_t)L * p->bank_elem;
    off = align_up(off + p->sz_bank, 256);
    p->off_tw = off;
    p->sz_tw = (size_t)L * p->tw_elem;
    off = align_up(off + p->sz_tw, 256);
    p->off_taps = off;
    p->sz_taps = (size_t)c.n_z * (size_t)c.n_taps * 16;
    off = align_up(off + p->sz_taps, 256);
    p->peak_tile_cap = (int64_t)c.n_z * ((c.max_bins + fdas::kPeakTileCols - 1) / fdas::kPeakTileCols);
    p->off_scr = off;
    p->sz_scr = fdas::peak_scratch_bytes(p->peak_tile_cap);
    off = align_up(off + p->sz_scr, 256);
    p->off_tab = off;
    if (c.compute == FDAS_FP8E4M3)   // FP32 staging of the bank, then one exponent per template
        p->sz_tab = fdas::fp8_staging_bytes(*p) + (size_t)c.n_z * sizeof(int32_t);
    else
        p->sz_tab = !p->mfma ? 0 : (L == fdas::m8k::kL ? fdas::m8k::kTableBytes : fdas::m4k::kTableBytes);
    off = align_up(off + p->sz_tab, 256);
    p->off_batch = off;
    p->batch_hdr = align_up((size_t)p->n_chunks * sizeof(int32_t), 256);   // one counter per template chunk
    p->sz_batch = c.max_jobs > 0 ? p->batch_hdr + (size_t)c.max_jobs * sizeof(fdas_batch_job) : 0;
    off = align_up(off + p->sz_batch, 256);
    p->ws_bytes = off;
    p->cfg.algo = p->mfma ? FDAS_ALGO_MFMA : FDAS_ALGO_VALU;

    *workspace_bytes = p->ws_bytes;
    *out = p;
    return FDAS_OK;
}

void fdas_destroy(fdas_plan_t plan) { delete plan; }

int fdas_set_workspace(fdas_plan_t p, void *dev, size_t bytes) {
    if (!p) return FDAS_E_INVALID;
    if (!dev) return FDAS_E_WORKSPACE;
    if (!aligned16(dev)) return FDAS_E_INVALID;
    if (bytes < p->ws_bytes) return FDAS_E_WORKSPACE;
    p->ws = dev;
    p->ws_size = bytes;
    p->templates_ready = false;
    p->batch_jobs = 0;
    return FDAS_OK;
}

int fdas_get_layout(fdas_plan_t p, fdas_layout *o) {
    if (!p || !o) return FDAS_E_INVALID;
    std::memset(o, 0, sizeof(*o));
    o->total_bytes = p->ws_bytes;
    o->bank_offset = p->off_bank;
    o->bank_bytes = p->sz_bank;
    o->twiddle_offset = p->off_tw;
    o->twiddle_bytes = p->sz_tw;
    o->scratch_offset = p->off_scr;
    o->scratch_bytes = p->sz_scr;
    o->seg_len = p->L;
    o->valid_per_seg = p->V;
    o->z_chunk = p->z_chunk;
    o->bank_elem_bytes = p->bank_elem;
    o->algo = p->cfg.algo;
    o->tables_offset = p->off_tab;
    o->tables_bytes = p->sz_tab;
    return FDAS_OK;
}

int fdas_make_templates(fdas_plan_t p, void *stream) {
    if (!p) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    const int s = hip_status(fdas::launch_make_templates(*p, static_cast<hipStream_t>(stream)));
    if (s == FDAS_OK) p->templates_ready = true;
    return s;
}

int fdas_make_templates_jerk(fdas_plan_t p, double w, void *stream) {
    if (!p || !std::isfinite(w)) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    p->templates_ready = false;
    const int s = hip_status(fdas::launch_make_templates(*p, static_cast<hipStream_t>(stream), w));
    if (s == FDAS_OK) p->templates_ready = true;
    return s;
}

int fdas_correlate(fdas_plan_t p, const void *spectrum, int64_t n_bins, void *plane, void *stream) {
    if (!p || !spectrum || !plane) return FDAS_E_INVALID;
    if (!aligned16(spectrum) || !aligned16(plane)) return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p->cfg.max_bins) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    if (!p->templates_ready) return FDAS_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->mfma && p->L == fdas::m4k::kL) return hip_status(fdas::launch_correlate_m4k(*p, spectrum, n_bins, plane, st));
    if (p->mfma) return hip_status(fdas::launch_correlate_mfma(*p, spectrum, n_bins, plane, st));
    return hip_status(fdas::launch_correlate(*p, spectrum, n_bins, plane, st));
}

int fdas_peaks(fdas_plan_t p, const void *plane, int64_t n_bins, float threshold, fdas_peak *out,
               int64_t capacity, int64_t *n_found, void *stream) {
    if (!p || !plane || !n_found || capacity < 0 || (capacity > 0 && !out)) return FDAS_E_INVALID;
    // the plane is read element by element: element alignment suffices (a
    // job's plane inside a batch buffer starts anywhere)
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(plane) % pe) != 0 || (out && !aligned16(out)) ||
        (reinterpret_cast<uintptr_t>(n_found) & 7u))
        return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p->cfg.max_bins) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    return hip_status(
        fdas::launch_peaks(*p, plane, n_bins, threshold, out, capacity, n_found, static_cast<hipStream_t>(stream)));
}

static bool prep_length_ok(int64_t n_t) { return fdas::prep_length_supported(n_t); }

int fdas_prepare_workspace(int64_t n_t, size_t *workspace_bytes) {
    if (!workspace_bytes) return FDAS_E_INVALID;
    if (n_t < 4) return FDAS_E_INVALID;
    if (!prep_length_ok(n_t)) return FDAS_E_UNSUPPORTED;
    *workspace_bytes = fdas::prep_workspace_bytes(n_t);
    return FDAS_OK;
}

int fdas_prepare(const float *series, int64_t n_t, void *spectrum, void *workspace, size_t workspace_bytes,
                 void *stream) {
    if (!series || !spectrum || n_t < 4) return FDAS_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(series) & 7u) || !aligned16(spectrum)) return FDAS_E_INVALID;
    if (!prep_length_ok(n_t)) return FDAS_E_UNSUPPORTED;
    if (!workspace || workspace_bytes < fdas::prep_workspace_bytes(n_t) || !aligned16(workspace))
        return FDAS_E_WORKSPACE;
    return hip_status(fdas::launch_prepare(series, n_t, spectrum, workspace, static_cast<hipStream_t>(stream)));
}

int fdas_band_max(fdas_plan_t p, const void *plane, int64_t n_bins, const int64_t *windows, int32_t n_windows,
                  fdas_peak *out, void *stream) {
    if (!p || !plane || !windows || !out) return FDAS_E_INVALID;
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(plane) % pe) != 0 || (reinterpret_cast<uintptr_t>(windows) & 7u) ||
        !aligned16(out))
        return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p->cfg.max_bins || n_windows < 1 || n_windows > 65535) return FDAS_E_INVALID;
    return hip_status(
        fdas::launch_band_max(*p, plane, n_bins, windows, n_windows, out, static_cast<hipStream_t>(stream)));
}

// The summing kernels address a plane row as one buffer resource with 32-bit
// byte offsets (plus the step between a thread's fundamentals): a row of
// n_bins values must stay below 4 GB less 1 MB.
static bool sum_rows_fit(const fdas_plan_s &p, int64_t n_bins) {
    return (uint64_t)n_bins * (uint64_t)(elem_bytes(p.cfg.plane_dtype) / 2) < 0xfff00000ull;
}

int fdas_harmonic_sum(fdas_plan_t p, const void *plane, int64_t n_bins, int32_t n_harm, void *out, void *stream) {
    if (!p || !plane || !out) return FDAS_E_INVALID;
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(plane) % pe) != 0 || (reinterpret_cast<uintptr_t>(out) % pe) != 0)
        return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p->cfg.max_bins || n_harm < 1 || n_harm > fdas::kMaxHarmonics)
        return FDAS_E_INVALID;
    if (p->cfg.n_z > 65535 || !sum_rows_fit(*p, n_bins)) return FDAS_E_UNSUPPORTED;
    return hip_status(fdas::launch_harmonic_sum(*p, plane, n_bins, n_harm, out, static_cast<hipStream_t>(stream)));
}

int fdas_harmonic_sums(fdas_plan_t p, const void *plane, int64_t n_bins, int32_t n_levels, const int32_t *n_harm,
                       void *const *outs, void *stream) {
    if (!p || !plane || !n_harm || !outs || n_levels < 1 || n_levels > 8) return FDAS_E_INVALID;
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(plane) % pe) != 0) return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p->cfg.max_bins) return FDAS_E_INVALID;
    for (int32_t l = 0; l < n_levels; ++l) {
        if (n_harm[l] < 1 || n_harm[l] > fdas::kMaxHarmonics || (l > 0 && n_harm[l] <= n_harm[l - 1]))
            return FDAS_E_INVALID;
        if (!outs[l] || (reinterpret_cast<uintptr_t>(outs[l]) % pe) != 0) return FDAS_E_INVALID;
    }
    if (p->cfg.n_z > 65535 || !sum_rows_fit(*p, n_bins)) return FDAS_E_UNSUPPORTED;
    return hip_status(fdas::launch_harmonic_sums(*p, plane, n_bins, n_levels, n_harm, outs, nullptr,
                                                 static_cast<hipStream_t>(stream)));
}

// Scratch of fdas_harmonic_sums_peaks: the peak finder's counters for the
// largest sum (shared by the sums, which are finished one after the other),
// then the tile and chunk flags of every sum back to back.
struct SumsPeakLayout {
    size_t work_bytes = 0, flags_off[8] = {}, total = 0;
    int64_t nh[8] = {}, n_cb[8] = {}, tiles[8] = {}, chunks[8] = {};
    bool fits = true;
};

static SumsPeakLayout sums_peak_layout(const fdas_plan_s &p, int64_t n_bins, int32_t n_levels, const int32_t *H) {
    SumsPeakLayout L;
    for (int32_t l = 0; l < n_levels; ++l) {
        L.nh[l] = (n_bins - 1) / H[l] + 1;
        L.n_cb[l] = (L.nh[l] + fdas::kPeakTileCols - 1) / fdas::kPeakTileCols;
        L.tiles[l] = L.n_cb[l] * p.cfg.n_z;
        L.chunks[l] = (L.tiles[l] + fdas::kPeakTilesPerChunk - 1) / fdas::kPeakTilesPerChunk;
        if (L.nh[l] > fdas::kMarkMaxBins || L.tiles[l] >= 0x7fffffffLL) L.fits = false;
    }
    L.work_bytes = align_up(fdas::peak_work_bytes(L.tiles[0]), 256);
    size_t off = L.work_bytes;
    for (int32_t l = 0; l < n_levels; ++l) {
        L.flags_off[l] = off;
        off += (size_t)(L.tiles[l] + L.chunks[l]);
    }
    L.total = align_up(off, 256);
    return L;
}

static int check_sums_list(const fdas_plan_s &p, int64_t n_bins, int32_t n_levels, const int32_t *n_harm) {
    if (!n_harm || n_levels < 1 || n_levels > 8) return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p.cfg.max_bins) return FDAS_E_INVALID;
    for (int32_t l = 0; l < n_levels; ++l)
        if (n_harm[l] < 1 || n_harm[l] > fdas::kMaxHarmonics || (l > 0 && n_harm[l] <= n_harm[l - 1]))
            return FDAS_E_INVALID;
    if (p.cfg.n_z > 65535 || !sum_rows_fit(p, n_bins)) return FDAS_E_UNSUPPORTED;
    return FDAS_OK;
}

static int check_sums_peaks_args(fdas_plan_t p, const void *plane, int64_t n_bins, int32_t n_levels,
                                 const int32_t *n_harm, void *const *outs, const float *thresholds,
                                 fdas_peak *const *peaks, int64_t capacity, const int64_t *n_found) {
    if (!p || !plane || !outs || !thresholds || !peaks || !n_found || capacity < 0) return FDAS_E_INVALID;
    const int s = check_sums_list(*p, n_bins, n_levels, n_harm);
    if (s != FDAS_OK) return s;
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(plane) % pe) != 0 || !aligned8(n_found)) return FDAS_E_INVALID;
    for (int32_t l = 0; l < n_levels; ++l) {
        if (!outs[l] || (reinterpret_cast<uintptr_t>(outs[l]) % pe) != 0) return FDAS_E_INVALID;
        if ((capacity > 0 && !peaks[l]) || (peaks[l] && !aligned16(peaks[l]))) return FDAS_E_INVALID;
    }
    return FDAS_OK;
}

// The sums with their peaks on a scratch region laid out by L: flags cleared
// by a kernel, sums stored with their tiles flagged, one finish per sum.
static hipError_t sums_peaks_on(const fdas_plan_s &p, const SumsPeakLayout &L, const void *plane, int64_t n_bins,
                                int32_t n_levels, const int32_t *n_harm, void *const *outs, const float *thresholds,
                                fdas_peak *const *peaks, int64_t capacity, int64_t *n_found, unsigned char *base,
                                hipStream_t st) {
    fdas::PeakMarks marks[8];
    for (int32_t l = 0; l < n_levels; ++l) {
        uint8_t *f = base + L.flags_off[l];
        marks[l] = fdas::make_peak_marks(f, f + L.tiles[l], L.n_cb[l], thresholds[l]);
    }
    hipError_t e = fdas::peak_flags_clear(base + L.flags_off[0], (int64_t)(L.total - L.flags_off[0]), st);
    if (e == hipSuccess) e = fdas::launch_harmonic_sums(p, plane, n_bins, n_levels, n_harm, outs, marks, st);
    for (int32_t l = 0; l < n_levels && e == hipSuccess; ++l)
        e = fdas::peaks_finish_plane(p, outs[l], L.nh[l], thresholds[l], marks[l].flags, marks[l].cflags, base,
                                     peaks[l], capacity, n_found + l, st);
    return e;
}

int fdas_harmonic_sums_peaks_workspace(fdas_plan_t p, int64_t n_bins, int32_t n_levels, const int32_t *n_harm,
                                       size_t *scratch_bytes) {
    if (!p || !scratch_bytes) return FDAS_E_INVALID;
    const int s = check_sums_list(*p, n_bins, n_levels, n_harm);
    if (s != FDAS_OK) return s;
    const SumsPeakLayout L = sums_peak_layout(*p, n_bins, n_levels, n_harm);
    if (!L.fits) return FDAS_E_UNSUPPORTED;
    *scratch_bytes = L.total;
    return FDAS_OK;
}

int fdas_harmonic_sums_peaks(fdas_plan_t p, const void *plane, int64_t n_bins, int32_t n_levels,
                             const int32_t *n_harm, void *const *outs, const float *thresholds,
                             fdas_peak *const *peaks, int64_t capacity, int64_t *n_found, void *scratch,
                             size_t scratch_bytes, void *stream) {
    const int s = check_sums_peaks_args(p, plane, n_bins, n_levels, n_harm, outs, thresholds, peaks, capacity,
                                        n_found);
    if (s != FDAS_OK) return s;
    const SumsPeakLayout L = sums_peak_layout(*p, n_bins, n_levels, n_harm);
    if (!L.fits) return FDAS_E_UNSUPPORTED;
    if (!scratch || !aligned16(scratch) || scratch_bytes < L.total) return FDAS_E_WORKSPACE;
    return hip_status(sums_peaks_on(*p, L, plane, n_bins, n_levels, n_harm, outs, thresholds, peaks, capacity,
                                    n_found, static_cast<unsigned char *>(scratch),
                                    static_cast<hipStream_t>(stream)));
}

int fdas_harmonic_sums_peaks_noalloc(fdas_plan_t p, const void *plane, int64_t n_bins, int32_t n_levels,
                                     const int32_t *n_harm, void *const *outs, const float *thresholds,
                                     fdas_peak *const *peaks, int64_t capacity, int64_t *n_found, void *stream) {
    const int s = check_sums_peaks_args(p, plane, n_bins, n_levels, n_harm, outs, thresholds, peaks, capacity,
                                        n_found);
    if (s != FDAS_OK) return s;
    const SumsPeakLayout L = sums_peak_layout(*p, n_bins, n_levels, n_harm);
    if (!L.fits) return FDAS_E_UNSUPPORTED;
    if (L.total > kNoallocScratchBytes) return FDAS_E_WORKSPACE;
    unsigned char *base = nullptr;
    const hipError_t e = noalloc_scratch(&base);
    if (e != hipSuccess) return hip_status(e);
    return hip_status(sums_peaks_on(*p, L, plane, n_bins, n_levels, n_harm, outs, thresholds, peaks, capacity,
                                    n_found, base, static_cast<hipStream_t>(stream)));
}

int fdas_harmonic_sum_peaks(fdas_plan_t p, const void *plane, int64_t n_bins, int32_t n_harm, void *out,
                            float threshold, fdas_peak *peaks, int64_t capacity, int64_t *n_found, void *stream) {
    if (!p || !plane || !out || !n_found || capacity < 0 || (capacity > 0 && !peaks)) return FDAS_E_INVALID;
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(plane) % pe) != 0 || (reinterpret_cast<uintptr_t>(out) % pe) != 0 ||
        (peaks && !aligned16(peaks)) || (reinterpret_cast<uintptr_t>(n_found) & 7u))
        return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p->cfg.max_bins || n_harm < 1 || n_harm > fdas::kMaxHarmonics)
        return FDAS_E_INVALID;
    if (p->cfg.n_z > 65535 || !sum_rows_fit(*p, n_bins)) return FDAS_E_UNSUPPORTED;
    if (!p->ws) return FDAS_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nh = (n_bins - 1) / n_harm + 1;
    const int64_t n_cb = (nh + fdas::kPeakTileCols - 1) / fdas::kPeakTileCols;
    if (nh > fdas::kMarkMaxBins || (int64_t)p->cfg.n_z * n_cb >= 0x7fffffffLL) {   // sum, then the streaming finder
        hipError_t e = fdas::launch_harmonic_sum(*p, plane, n_bins, n_harm, out, st);
        if (e == hipSuccess) e = fdas::launch_peaks(*p, out, nh, threshold, peaks, capacity, n_found, st);
        return hip_status(e);
    }
    fdas::PeakMarks m;
    hipError_t e = fdas::peak_marks(*p, nh, threshold, &m, st);
    if (e == hipSuccess) e = fdas::launch_harmonic_sum_marked(*p, plane, n_bins, n_harm, out, m, st);
    if (e == hipSuccess) e = fdas::launch_peaks(*p, out, nh, threshold, peaks, capacity, n_found, st, true);
    return hip_status(e);
}

int fdas_set_batch(fdas_plan_t p, const fdas_job *jobs, int32_t n_jobs, int64_t spectra_bins, int64_t plane_cells,
                   void *stream) {
    if (!p || !jobs || n_jobs < 1) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    p->batch_jobs = 0;
    if (n_jobs > p->cfg.max_jobs) return FDAS_E_INVALID;
    std::vector<fdas_batch_job> tab((size_t)n_jobs);
    int64_t segs = 0, tiles = 0, chunks = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const fdas_job &j = jobs[i];
        if (j.n_bins < 1 || j.n_bins > p->cfg.max_bins || j.spec_off < 0 || j.plane_off < 0) return FDAS_E_INVALID;
        if (j.spec_off > spectra_bins - j.n_bins) return FDAS_E_INVALID;
        if (j.n_bins > (plane_cells - j.plane_off) / p->cfg.n_z || j.plane_off > plane_cells) return FDAS_E_INVALID;
        tab[i] = {j.spec_off, j.n_bins, j.plane_off, segs, tiles, chunks};
        segs += (j.n_bins + p->V - 1) / p->V;
        // peak tiles of the job's plane, and their chunks (batched peak finding)
        const int64_t jt = (int64_t)p->cfg.n_z * ((j.n_bins + fdas::kPeakTileCols - 1) / fdas::kPeakTileCols);
        tiles += jt;
        chunks += (jt + fdas::kPeakTilesPerChunk - 1) / fdas::kPeakTilesPerChunk;
        // segment and tile indices are 32-bit on the device; each chunk's
        // counter overshoots the segment count by at most one per workgroup
        if (segs * p->n_chunks > 0x7fffffffLL - (1 << 20)) return FDAS_E_INVALID;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(static_cast<unsigned char *>(p->ws) + p->off_batch + p->batch_hdr, tab.data(),
                                  tab.size() * sizeof(fdas_batch_job), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e);
    p->batch_host = std::move(tab);
    p->batch_jobs = n_jobs;
    p->batch_tiles = segs * p->n_chunks;
    p->batch_peak_tiles = tiles;
    p->batch_peak_chunks = chunks;
    return FDAS_OK;
}

int fdas_correlate_batch(fdas_plan_t p, const void *spectra, void *planes, void *stream) {
    if (!p || !spectra || !planes) return FDAS_E_INVALID;
    if (!aligned16(spectra) || !aligned16(planes)) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    if (!p->templates_ready || p->batch_jobs < 1) return FDAS_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->mfma && p->L == fdas::m4k::kL) return hip_status(fdas::launch_correlate_m4k_batch(*p, spectra, planes, st));
    const size_t pe = p->cfg.plane_dtype == FDAS_FP64 ? 8 : p->cfg.plane_dtype == FDAS_FP32 ? 4 : 2;
    for (const fdas_batch_job &j : p->batch_host) {
        const void *sp = static_cast<const unsigned char *>(spectra) + (size_t)j.spec_off * 8;
        void *pl = static_cast<unsigned char *>(planes) + (size_t)j.plane_off * pe;
        const hipError_t e = p->mfma ? fdas::launch_correlate_mfma(*p, sp, j.n_bins, pl, st)
                                     : fdas::launch_correlate(*p, sp, j.n_bins, pl, st);
        if (e != hipSuccess) return hip_status(e);
    }
    return FDAS_OK;
}


// The marking correlation indexes columns and tiles in 32 bits.
static bool mark_fits(const fdas_plan_s &p, int64_t n_bins) {
    const int64_t n_cb = (n_bins + fdas::kPeakTileCols - 1) / fdas::kPeakTileCols;
    return p.mfma && p.L == fdas::m4k::kL && n_bins <= fdas::kMarkMaxBins && (int64_t)p.cfg.n_z * n_cb < 0x7fffffffLL;
}

int fdas_correlate_peaks(fdas_plan_t p, const void *spectrum, int64_t n_bins, void *plane, float threshold,
                         fdas_peak *out, int64_t capacity, int64_t *n_found, void *stream) {
    if (!p || !spectrum || !plane || !n_found || capacity < 0 || (capacity > 0 && !out)) return FDAS_E_INVALID;
    if (!aligned16(spectrum) || !aligned16(plane) || (out && !aligned16(out)) || !aligned8(n_found))
        return FDAS_E_INVALID;
    if (n_bins < 1 || n_bins > p->cfg.max_bins) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    if (!p->templates_ready) return FDAS_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (mark_fits(*p, n_bins)) {
        fdas::PeakMarks m;
        hipError_t e = fdas::peak_marks(*p, n_bins, threshold, &m, st);
        if (e == hipSuccess) e = fdas::launch_correlate_m4k_marked(*p, spectrum, n_bins, plane, m, st);
        if (e == hipSuccess) e = fdas::launch_peaks(*p, plane, n_bins, threshold, out, capacity, n_found, st, true);
        return hip_status(e);
    }
    const int s = fdas_correlate(p, spectrum, n_bins, plane, stream);
    if (s != FDAS_OK) return s;
    return hip_status(fdas::launch_peaks(*p, plane, n_bins, threshold, out, capacity, n_found, st));
}

int fdas_batch_peaks_workspace(fdas_plan_t p, size_t *scratch_bytes) {
    if (!p || !scratch_bytes) return FDAS_E_INVALID;
    if (p->batch_jobs < 1) return FDAS_E_STATE;
    *scratch_bytes = fdas::batch_peak_scratch_bytes(*p);
    return FDAS_OK;
}

int fdas_correlate_batch_peaks(fdas_plan_t p, const void *spectra, void *planes, float threshold, fdas_peak *out,
                               int64_t capacity, int64_t *n_found, void *scratch, size_t scratch_bytes,
                               void *stream) {
    if (!p || !spectra || !planes || !n_found || capacity < 0 || (capacity > 0 && !out)) return FDAS_E_INVALID;
    if (!aligned16(spectra) || !aligned16(planes) || (out && !aligned16(out)) || !aligned8(n_found))
        return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    if (!p->templates_ready || p->batch_jobs < 1) return FDAS_E_STATE;
    if (!scratch || !aligned16(scratch) || scratch_bytes < fdas::batch_peak_scratch_bytes(*p))
        return FDAS_E_WORKSPACE;
    if (capacity > 0 && p->batch_jobs > INT64_MAX / capacity) return FDAS_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(stream);
    fdas::PeakMarks m;
    hipError_t e = fdas::batch_peak_marks(*p, scratch, threshold, &m, st);
    if (e != hipSuccess) return hip_status(e);
    if (mark_fits(*p, p->cfg.max_bins)) {
        e = fdas::launch_correlate_m4k_batch_marked(*p, spectra, planes, m, st);
    } else {
        const int s = fdas_correlate_batch(p, spectra, planes, stream);
        if (s != FDAS_OK) return s;
        e = fdas::batch_peak_mark_pass(*p, planes, m, st);
    }
    if (e == hipSuccess) e = fdas::batch_peaks_finish(*p, planes, scratch, threshold, out, capacity, n_found, st);
    return hip_status(e);
}

static bool sum_levels_ok(int32_t n_levels, const int32_t *n_harm) {
    if (!n_harm || n_levels < 1 || n_levels > 8) return false;
    for (int32_t l = 0; l < n_levels; ++l)
        if (n_harm[l] < 1 || n_harm[l] > fdas::kMaxHarmonics || (l > 0 && n_harm[l] <= n_harm[l - 1])) return false;
    return true;
}

// The stored batch as the jobs of a batch harmonic-sums call.
static fdas::SumBatch plan_batch(const fdas_plan_s &p) {
    return fdas::SumBatch{p.batch_host.data(), p.batch_jobs,
                          reinterpret_cast<const fdas_batch_job *>(static_cast<const unsigned char *>(p.ws) +
                                                                   p.off_batch + p.batch_hdr)};
}

static int check_sum_layout(const fdas::BatchSumsLayout &L) {
    return L.blocks > 0x7fffffffLL || L.tiles >= 0x7fffffffLL ? FDAS_E_UNSUPPORTED : FDAS_OK;
}

static int check_batch_sums(fdas_plan_t p, int32_t n_levels, const int32_t *n_harm) {
    if (!p || !sum_levels_ok(n_levels, n_harm)) return FDAS_E_INVALID;
    if (p->batch_jobs < 1) return FDAS_E_STATE;
    if (p->cfg.n_z > 65535 || p->batch_jobs > 32767 || !sum_rows_fit(*p, p->cfg.max_bins)) return FDAS_E_UNSUPPORTED;
    return check_sum_layout(fdas::batch_sums_layout(*p, plan_batch(*p), n_levels, n_harm));
}

int fdas_batch_harmonic_sums_peaks_workspace(fdas_plan_t p, int32_t n_levels, const int32_t *n_harm,
                                             size_t *scratch_bytes) {
    if (!scratch_bytes) return FDAS_E_INVALID;
    const int s = check_batch_sums(p, n_levels, n_harm);
    if (s != FDAS_OK) return s;
    *scratch_bytes = fdas::batch_sums_layout(*p, plan_batch(*p), n_levels, n_harm).bytes;
    return FDAS_OK;
}

int fdas_batch_harmonic_sums_peaks(fdas_plan_t p, const void *planes, int32_t n_levels, const int32_t *n_harm,
                                   const float *thresholds, fdas_peak *peaks, int64_t capacity, int64_t *n_found,
                                   void *scratch, size_t scratch_bytes, void *stream) {
    const int s = check_batch_sums(p, n_levels, n_harm);
    if (s != FDAS_OK) return s;
    if (!planes || !thresholds || !n_found || capacity < 0 || (capacity > 0 && !peaks)) return FDAS_E_INVALID;
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(planes) % pe) != 0 || (peaks && !aligned16(peaks)) || !aligned8(n_found))
        return FDAS_E_INVALID;
    const fdas::SumBatch b = plan_batch(*p);
    const fdas::BatchSumsLayout L = fdas::batch_sums_layout(*p, b, n_levels, n_harm);
    if (capacity > 0 && L.lists > INT64_MAX / capacity) return FDAS_E_INVALID;
    if (!p->ws) return FDAS_E_WORKSPACE;
    if (!scratch || !aligned16(scratch) || scratch_bytes < L.bytes) return FDAS_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = fdas::launch_batch_sums_mark(*p, b, L, planes, n_levels, n_harm, thresholds, scratch, st);
    if (e == hipSuccess) e = fdas::batch_sums_finish(*p, b, L, planes, scratch, peaks, capacity, n_found, st);
    return hip_status(e);
}

// fdas_harmonic_peaks: the plane as a batch of one job, its record in the
// first 256 bytes of the scratch, the batch layout after it.
static constexpr size_t kOneJobBytes = 256;
static_assert(sizeof(fdas_batch_job) <= kOneJobBytes, "one job record");

static int check_harmonic_peaks(fdas_plan_t p, int64_t n_bins, int32_t n_levels, const int32_t *n_harm,
                                fdas_batch_job *job, fdas::BatchSumsLayout *L) {
    if (!p || !sum_levels_ok(n_levels, n_harm) || n_bins < 1 || n_bins > p->cfg.max_bins) return FDAS_E_INVALID;
    if (p->cfg.n_z > 65535 || !sum_rows_fit(*p, n_bins)) return FDAS_E_UNSUPPORTED;
    *job = fdas_batch_job{0, n_bins, 0, 0, 0, 0};
    *L = fdas::batch_sums_layout(*p, fdas::SumBatch{job, 1, nullptr}, n_levels, n_harm);
    return check_sum_layout(*L);
}

int fdas_harmonic_peaks_workspace(fdas_plan_t p, int64_t n_bins, int32_t n_levels, const int32_t *n_harm,
                                  size_t *scratch_bytes) {
    if (!scratch_bytes) return FDAS_E_INVALID;
    fdas_batch_job job;
    fdas::BatchSumsLayout L;
    const int s = check_harmonic_peaks(p, n_bins, n_levels, n_harm, &job, &L);
    if (s != FDAS_OK) return s;
    *scratch_bytes = kOneJobBytes + L.bytes;
    return FDAS_OK;
}

int fdas_harmonic_peaks(fdas_plan_t p, const void *plane, int64_t n_bins, int32_t n_levels, const int32_t *n_harm,
                        const float *thresholds, fdas_peak *peaks, int64_t capacity, int64_t *n_found, void *scratch,
                        size_t scratch_bytes, void *stream) {
    fdas_batch_job job;
    fdas::BatchSumsLayout L;
    const int s = check_harmonic_peaks(p, n_bins, n_levels, n_harm, &job, &L);
    if (s != FDAS_OK) return s;
    if (!plane || !thresholds || !n_found || capacity < 0 || (capacity > 0 && !peaks)) return FDAS_E_INVALID;
    const uintptr_t pe = (uintptr_t)elem_bytes(p->cfg.plane_dtype) / 2;   // one real value
    if ((reinterpret_cast<uintptr_t>(plane) % pe) != 0 || (peaks && !aligned16(peaks)) || !aligned8(n_found))
        return FDAS_E_INVALID;
    if (capacity > 0 && L.lists > INT64_MAX / capacity) return FDAS_E_INVALID;
    if (!scratch || !aligned16(scratch) || scratch_bytes < kOneJobBytes + L.bytes) return FDAS_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto *dev_job = static_cast<fdas_batch_job *>(scratch);
    const fdas::SumBatch b{&job, 1, dev_job};
    unsigned char *rest = static_cast<unsigned char *>(scratch) + kOneJobBytes;
    hipError_t e = fdas::write_one_job(dev_job, n_bins, st);
    if (e == hipSuccess) e = fdas::launch_batch_sums_mark(*p, b, L, plane, n_levels, n_harm, thresholds, rest, st);
    if (e == hipSuccess) e = fdas::batch_sums_finish(*p, b, L, plane, rest, peaks, capacity, n_found, st);
    return hip_status(e);
}

int fdas_refine(const void *spectrum, int64_t n_bins, int32_t n_cand, double *r, double *z, double *power,
                double *dp_dr, double *dp_dz, int32_t taps, int32_t n_steps, double eta_r_scale, double eta_z_scale,
                void *stream) {
    if (!spectrum || n_bins < 1 || n_cand < 0 || n_steps < 0) return FDAS_E_INVALID;
    if (taps < 2 || taps > 64 || (taps & 1)) return FDAS_E_INVALID;
    if (n_cand > 0 && (!r || !z)) return FDAS_E_INVALID;
    if (!aligned8(spectrum) || !aligned8(r) || !aligned8(z) || !aligned8(power) || !aligned8(dp_dr) ||
        !aligned8(dp_dz))
        return FDAS_E_INVALID;
    if (!std::isfinite(eta_r_scale) || !std::isfinite(eta_z_scale)) return FDAS_E_INVALID;
    return hip_status(fdas::launch_refine(spectrum, n_bins, n_cand, r, z, power, dp_dr, dp_dz, taps, n_steps,
                                          eta_r_scale, eta_z_scale, static_cast<hipStream_t>(stream)));
}

int fdas_refine_backward(const void *spectrum, int64_t n_bins, int32_t n_cand, const double *r, const double *z,
                         const double *grad_power, double *grad_r, double *grad_z, int32_t taps, void *stream) {
    if (!spectrum || n_bins < 1 || n_cand < 0) return FDAS_E_INVALID;
    if (taps < 2 || taps > 64 || (taps & 1)) return FDAS_E_INVALID;
    if (n_cand > 0 && (!r || !z || !grad_power || !grad_r || !grad_z)) return FDAS_E_INVALID;
    if (!aligned8(spectrum) || !aligned8(r) || !aligned8(z) || !aligned8(grad_power) || !aligned8(grad_r) ||
        !aligned8(grad_z))
        return FDAS_E_INVALID;
    return hip_status(fdas::launch_refine_backward(spectrum, n_bins, n_cand, r, z, grad_power, grad_r, grad_z, taps,
                                                   static_cast<hipStream_t>(stream)));
}

}  // extern "C"
