// Internal declarations shared by the libfdas translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/fdas.h"

namespace fdas {

// FDAS_OK for hipSuccess, else FDAS_E_HIP with the code kept for fdas_last_hip_error.
int hip_status_of(hipError_t e);

constexpr int kPointsPerThread = 16;   // complex points each thread keeps in registers
constexpr int kMinLog2L = 10;
constexpr int kMaxLog2L = 14;

}  // namespace fdas

// One job of a batched launch as the device sees it (offsets in elements).
struct fdas_batch_job {
    int64_t spec_off;     // first bin of the job's spectrum in the spectra buffer
    int64_t n_bins;       // its length N
    int64_t plane_off;    // first cell of its n_z x N plane in the planes buffer
    int64_t seg_base;     // index of its first segment among all jobs' segments
    int64_t tile_base;    // its first peak tile among all jobs' tiles (batched peak finding)
    int64_t chunk_base;   // its first chunk of peak tiles among all jobs' chunks
};

struct fdas_plan_s {
    fdas_config cfg;
    int32_t L = 0, log2L = 0, M = 0, V = 0;
    int32_t z_chunk = 0, n_chunks = 0;
    int32_t bank_elem = 0;       // bytes per complex template value
    int32_t tw_elem = 0;         // bytes per complex twiddle
    size_t ws_bytes = 0;
    size_t off_bank = 0, sz_bank = 0;
    size_t off_tw = 0, sz_tw = 0;
    size_t off_taps = 0, sz_taps = 0;      // FP64 taps, n_z x M complex (template build)
    size_t off_scr = 0, sz_scr = 0;        // peak counters
    size_t off_tab = 0, sz_tab = 0;        // matrix-core operator/twiddle tables
    bool mfma = false;                     // matrix-core correlation kernel (L = 4096 or 8192)
    size_t off_batch = 0, sz_batch = 0;    // per-chunk segment counters (batch_hdr B) + job table
    size_t batch_hdr = 0;
    int32_t batch_jobs = 0;                // jobs set by fdas_set_batch (0: none)
    int64_t batch_tiles = 0;
    int64_t batch_peak_tiles = 0;          // peak tiles of all jobs' planes
    int64_t batch_peak_chunks = 0;         // chunks of peak tiles of all jobs' planes
    std::vector<fdas_batch_job> batch_host;   // host copy of the job table
    int64_t peak_tile_cap = 0;             // number of peak tiles the scratch holds
    void *ws = nullptr;
    size_t ws_size = 0;
    bool templates_ready = false;
};

namespace fdas {

// Template bank + twiddle table (templates.hip).
hipError_t launch_make_templates(const fdas_plan_s &p, hipStream_t s, double w = 0.0);

// Matrix-core correlation, L = 8192, BF16 form (correlate_mfma.hip).
hipError_t launch_correlate_mfma(const fdas_plan_s &p, const void *spec, int64_t n,
                                 void *plane, hipStream_t s);

// Matrix-core correlation, L = 4096, BF16 form (correlate_m4k.hip).
hipError_t launch_correlate_m4k(const fdas_plan_s &p, const void *spec, int64_t n,
                                void *plane, hipStream_t s);

hipError_t launch_correlate_m4k_batch(const fdas_plan_s &p, const void *spectra, void *planes, hipStream_t s);

// Resets the n per-chunk segment counters of a batch (batch.hip); a kernel,
// so graph capture records no memset.
__global__ void k_batch_reset(int32_t *counters, int32_t n);

struct PeakMarks;

// L = 4096 matrix-core correlation that also marks the peak tiles of cells
// above a threshold while storing the plane (marks: the flags of this plane;
// batch: the flags of all jobs, each job at its tile_base / chunk_base).
hipError_t launch_correlate_m4k_marked(const fdas_plan_s &p, const void *spec, int64_t n, void *plane,
                                       const PeakMarks &marks, hipStream_t s);
hipError_t launch_correlate_m4k_batch_marked(const fdas_plan_s &p, const void *spectra, void *planes,
                                             const PeakMarks &marks, hipStream_t s);

// Correlation (correlate.hip).
// FP8 (e4m3) form: bytes of the FP32 bank staging at the start of the tables
// region (the per-template exponents follow it), the bank conversion and the
// correlation.
size_t fp8_staging_bytes(const fdas_plan_s &p);
hipError_t launch_fp8_bank(const fdas_plan_s &p, hipStream_t st);
hipError_t launch_correlate_fp8(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st);
hipError_t launch_correlate(const fdas_plan_s &p, const void *spec, int64_t n,
                            void *plane, hipStream_t s);

// Refinement (refine.hip).
hipError_t launch_refine(const void *spec, int64_t n, int32_t n_cand, double *r, double *z, double *power,
                         double *dp_dr, double *dp_dz, int32_t taps, int32_t n_steps, double s_r, double s_z,
                         hipStream_t st);
hipError_t launch_refine_backward(const void *spec, int64_t n, int32_t n_cand, const double *r, const double *z,
                                  const double *grad_p, double *grad_r, double *grad_z, int32_t taps, hipStream_t st);

// Peaks (peaks.hip).
constexpr int kPeakTileCols = 1024;     // columns per peak tile (one row per tile)
constexpr int kPeakTilesPerChunk = 16;  // tiles per chunk (unit of the per-chunk totals and offsets)
size_t peak_scratch_bytes(int64_t n_tiles);
// premarked: the tile flags of this plane were set by peak_marks + a marking
// correlation (the clear and the streaming mark pass are skipped)
hipError_t launch_peaks(const fdas_plan_s &p, const void *plane, int64_t n, float thr,
                        fdas_peak *out, int64_t capacity, int64_t *n_found, hipStream_t s,
                        bool premarked = false);
// Zeroes the tile flags of an n-bin plane in the plan's scratch and describes
// them for a marking correlation.
hipError_t peak_marks(const fdas_plan_s &p, int64_t n, float thr, PeakMarks *marks, hipStream_t s);
// Batched peak finding over every job of the plan's batch, in a caller
// scratch of batch_peak_scratch_bytes: zero the flags (batch_peak_marks),
// mark them (a marking batch correlation, or batch_peak_mark_pass over the
// planes), then batch_peaks_finish: job i's peaks at out + i * capacity
// (job = i), its count at n_found[i].
size_t batch_peak_scratch_bytes(const fdas_plan_s &p);
// Count, scan and write of one n-bin plane whose tile flags (flags, cflags)
// a marking kernel set; counters in caller memory of peak_work_bytes(tiles).
size_t peak_work_bytes(int64_t n_tiles);
hipError_t peaks_finish_plane(const fdas_plan_s &p, const void *plane, int64_t n, float thr, const uint8_t *flags,
                              const uint8_t *cflags, void *work, fdas_peak *out, int64_t capacity, int64_t *n_found,
                              hipStream_t s);
// Zeroes n bytes of tile and chunk flags (a kernel: graph-capturable).
hipError_t peak_flags_clear(uint8_t *flags, int64_t n, hipStream_t s);
hipError_t batch_peak_marks(const fdas_plan_s &p, void *scratch, float thr, PeakMarks *marks, hipStream_t s);
hipError_t batch_peak_mark_pass(const fdas_plan_s &p, const void *planes, const PeakMarks &marks, hipStream_t s);
hipError_t batch_peaks_finish(const fdas_plan_s &p, const void *planes, void *scratch, float thr, fdas_peak *out,
                              int64_t capacity, int64_t *n_found, hipStream_t s);

// Spectrum preparation (prep.hip).
size_t prep_workspace_bytes(int64_t n_t);
// Series lengths fdas_prepare handles: 2^a (4 <= n_t <= 2^28) and 3 * 2^a (the
// four-step form: 3 * 2^7 <= n_t <= 3 * 2^22).
bool prep_length_supported(int64_t n_t);
hipError_t launch_prepare(const float *series, int64_t n_t, void *out, void *ws, hipStream_t st);

// Band maxima (bands.hip).
hipError_t launch_band_max(const fdas_plan_s &p, const void *plane, int64_t n, const int64_t *windows,
                           int32_t n_windows, fdas_peak *out, hipStream_t st);

// Harmonic summing (harmonic.hip).
constexpr int kMaxHarmonics = 32;
hipError_t launch_harmonic_sum(const fdas_plan_s &p, const void *plane, int64_t n, int n_harm, void *out,
                               hipStream_t st);
// Sums for an increasing list of n_levels (<= 8) harmonic counts in one
// pass, sum l to outs[l]; marks (n_levels entries) or null: the peak tiles
// of each sum flagged while it is stored.
// Harmonic sums of every job of a stored batch with their thresholded
// peaks, the sums never stored (harmonic.hip marks, peaks.hip finishes).
// Caller scratch layout (byte offsets, 256-aligned regions).
constexpr int kBatchPeakGrid = 2048;   // workgroups of the count and write kernels
// Chunk ranges of the count and write kernels: the chunks are cut into at
// most this many ranges, workgroup b taking ranges b, b + kBatchPeakGrid, ...
// (tiles that may hold peaks cluster where a bright signal is, so short
// ranges spread them over many workgroups); one total and one offset each.
constexpr int kPeakRanges = 32768;
struct BatchSumsLayout {
    int64_t tiles = 0, chunks = 0, blocks = 0, lists = 0;
    int hmax = 0;
    size_t off_counts = 0, off_block_counts = 0, off_wg_totals = 0, off_wg_offsets = 0, off_prefix = 0;
    size_t off_totals = 0, off_lists = 0, off_rows = 0, off_units = 0, clear_bytes = 0, bytes = 0;
};
// The jobs a batch harmonic-sums call covers: the host copy (for the
// layout) and the device table (for the kernels); a single plane is a batch
// of one job whose record the caller's scratch holds.
struct SumBatch {
    const fdas_batch_job *host;
    int32_t n_jobs;
    const fdas_batch_job *dev;
};
BatchSumsLayout batch_sums_layout(const fdas_plan_s &p, const SumBatch &b, int n_levels, const int32_t *H);
hipError_t launch_batch_sums_mark(const fdas_plan_s &p, const SumBatch &b, const BatchSumsLayout &L,
                                  const void *planes, int n_levels, const int32_t *H, const float *thr, void *scratch,
                                  hipStream_t s);
hipError_t batch_sums_finish(const fdas_plan_s &p, const SumBatch &b, const BatchSumsLayout &L, const void *planes,
                             void *scratch, fdas_peak *out, int64_t capacity, int64_t *n_found, hipStream_t s);
// Writes the one-job record {n_bins = n, everything else 0} to dev (a
// kernel, so graph capture records no copy from host memory).
hipError_t write_one_job(fdas_batch_job *dev, int64_t n, hipStream_t s);
hipError_t launch_harmonic_sums(const fdas_plan_s &p, const void *plane, int64_t n, int n_levels, const int32_t *H,
                                void *const *outs, const PeakMarks *marks, hipStream_t st);
// The same, also marking the peak tiles of the summed plane (marks from
// peak_marks for its (n - 1) / n_harm + 1 bins).
hipError_t launch_harmonic_sum_marked(const fdas_plan_s &p, const void *plane, int64_t n, int n_harm, void *out,
                                      const PeakMarks &marks, hipStream_t st);

}  // namespace fdas
