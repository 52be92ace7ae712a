/*
 * fdas.h -- C ABI of libfdas, the Fourier Domain Acceleration Search (FDAS)
 * hot path on AMD Instinct MI355X (gfx950).
 *
 * What is computed.  A binary pulsar's pulse frequency drifts linearly over
 * an observation of length T; its drift in Fourier bins is z = fdot T^2 and
 * its acceleration a = z c / (f T^2) (Eq. 1).  FDAS correlates the normalised
 * complex spectrum X[k], k in [0, N), with a bank of acceleration templates,
 * one per z on a grid, and the |.|^2 of the result is the f-fdot plane, on
 * which a pulsar shows as a peak with harmonics at integer multiples of f and
 * fdot (Section "Detailed explanation").  The correlation uses the
 * convolution theorem with overlap-save: the spectrum is cut into windows,
 * each window is transformed, multiplied by each template's transform,
 * inverse transformed, and the central part of each window is kept while the
 * contaminated edges are discarded (Section "Detailed explanation" and the
 * overlap-save flowchart figure there).
 *
 * Definitions used by every call (the paper prints no template formula; it
 * cites Ransom et al. 2002 for the method, Section "Introduction"):
 *   response   A(q, z) = int_0^1 exp(i pi (2 q u + z u^2)) du
 *   z grid     z_j = z_min + j * z_step, j in [0, n_z)
 *   taps       g_j[m] = conj(A(m - z_j/2, z_j)) / ||.||_2,  m in [-M/2, M/2)
 *              (r is the mean Fourier frequency; unit l2 norm after truncation)
 *   plane      P[j, r] = | sum_m X[r - m] g_j[m] |^2,  r in [0, N),
 *              with X = 0 outside [0, N)
 * Overlap-save with segment length L (power of two, L > M) keeps V = L - M
 * outputs per segment; segment s reads X[s V - M/2 .. s V - M/2 + L).  The
 * plane does not depend on L except through rounding.
 *
 * Precision forms (Section "Updating the pipeline to bfloat16"):
 *   FDAS_FP32  single precision throughout.
 *   FDAS_BF16  segment spectra, templates and transform stages stored in
 *              bfloat16 (round to nearest even), arithmetic accumulated in
 *              single precision.  The spectrum input stays single precision
 *              (the paper keeps its real FFT in single precision).
 *   FDAS_FP8E4M3  one step below bfloat16 (no FP8 form in the paper): the
 *              stored transform stages, the segment spectrum and the templates
 *              are OCP e4m3 (3 mantissa bits, largest 448) with power-of-two
 *              scales; each stored stage takes the largest scale that keeps the
 *              workgroup's largest component within 448, each template its
 *              own.  Arithmetic is single precision; the window is read in
 *              single precision.  Vector-ALU kernel, L in {1024, 2048, 4096}
 *              (0 chooses 4096); the e4m3 format has no infinities, so an Inf
 *              input turns its segments' outputs into NaN.
 *   FDAS_FP64  double precision throughout: the gold-standard plane.
 * Plane dtypes: FDAS_FP32 (4 B/cell), FDAS_BF16 (2 B/cell raw bfloat16; a
 * consumer widens it exactly to single precision by placing the two bytes in
 * the high half of a zeroed 32-bit word, Section "Casting between
 * single-precision and bfloat16"), FDAS_FP64 (8 B/cell, FP64 compute only).
 *
 * Conventions for every call:
 *   Memory    the library owns only the opaque plan.  Every device buffer
 *             (spectrum, plane, workspace, peak list) is allocated and owned
 *             by the caller and must stay alive until the stream work that
 *             uses it has finished.
 *   Streams   calls that take a stream enqueue asynchronous work on it (NULL
 *             = the null stream) and never synchronise the device; a plan is
 *             used from one stream at a time.
 *   Status    calls return FDAS_OK (0) or a negative fdas_status; nothing
 *             throws across the ABI.  FDAS_E_HIP keeps the HIP error code,
 *             readable through fdas_last_hip_error().
 *   Alignment device pointers must be 16-byte aligned (FDAS_E_INVALID).
 *   NaN/Inf   propagate; an Inf or NaN anywhere in a segment pollutes every
 *             output of that segment after the inverse transform (Section
 *             "IEEE-754 Half vs bfloat16 precision").  No checks on the hot
 *             path.
 */
#ifndef FDAS_H
#define FDAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdas_plan_s *fdas_plan_t;

typedef enum {
    FDAS_FP32 = 0,
    FDAS_BF16 = 1,
    FDAS_FP8E4M3 = 2,   /* OCP e4m3 storage form (vector-ALU kernel, L <= 4096) */
    FDAS_FP64 = 3
} fdas_dtype;

typedef enum {
    FDAS_OK = 0,
    FDAS_E_INVALID = -1,      /* bad argument or configuration */
    FDAS_E_WORKSPACE = -2,    /* no workspace, or workspace too small */
    FDAS_E_HIP = -3,          /* a HIP runtime call failed */
    FDAS_E_CAPACITY = -4,     /* more peaks than the output can hold */
    FDAS_E_UNSUPPORTED = -5,  /* valid request this build does not implement */
    FDAS_E_STATE = -6         /* call out of order (e.g. correlate before templates) */
} fdas_status;

typedef struct {
    int64_t max_bins;     /* N: largest spectrum length (complex bins) the plan serves */
    double  z_min;        /* first template drift (bins) */
    double  z_step;       /* template spacing (bins), > 0 unless n_z == 1 */
    int32_t n_z;          /* number of templates, >= 1 */
    int32_t n_taps;       /* M: even, >= 2; the overlap between segments */
    int32_t seg_len;      /* L: power of two in [1024, 16384], L > M; 0 = choose (BF16: 4096 for
                             M <= 512, 8192 for M <= 2048; FP8: 4096; otherwise the power of
                             two >= 8 M, at least 1024, at most 8192 for FP64) */
    int32_t compute;      /* FDAS_FP32 | FDAS_BF16 | FDAS_FP8E4M3 | FDAS_FP64 */
    int32_t plane_dtype;  /* FDAS_FP32 | FDAS_BF16 (not with FP64 compute) | FDAS_FP64 (FP64 compute only) */
    int32_t z_chunk;      /* templates per workgroup; 0 = choose */
    int32_t algo;         /* FDAS_ALGO_AUTO | FDAS_ALGO_VALU | FDAS_ALGO_MFMA */
    int32_t max_jobs;     /* largest batch fdas_set_batch accepts (0: batches unused) */
} fdas_config;

/* Kernel family of the correlation.  AUTO picks the matrix-core kernel where
 * one exists (BF16 compute with L = 4096 or 8192) and the vector-ALU kernel
 * otherwise; MFMA on a configuration without a matrix-core kernel is
 * FDAS_E_UNSUPPORTED.  Both compute the same plane (the MFMA kernel rounds
 * its DFT operators to bfloat16 as well). */
typedef enum { FDAS_ALGO_AUTO = 0, FDAS_ALGO_VALU = 1, FDAS_ALGO_MFMA = 2 } fdas_algo;

/* One spectrum of a batch (offsets in elements): its n_bins complex64 bins
 * start at spectra[spec_off], its n_z x n_bins plane (row stride n_bins) at
 * planes[plane_off]. */
typedef struct {
    int64_t spec_off;
    int64_t n_bins;
    int64_t plane_off;
} fdas_job;

/* One entry of a peak list (24 bytes).  r is the spectral bin, z_idx the
 * template row, power the plane value widened to single precision. */
typedef struct {
    int64_t r;
    int32_t z_idx;
    int32_t job;
    float   power;
    float   reserved;
} fdas_peak;

/* Workspace layout of a plan, byte offsets from the workspace base. */
typedef struct {
    size_t total_bytes;
    size_t bank_offset;      /* template bank: n_z x L complex, compute dtype; natural bin order for
                                the vector-ALU kernel, matrix-core lane order for the MFMA kernel */
    size_t bank_bytes;
    size_t twiddle_offset;   /* exp(-2 pi i e / L), e in [0, L), compute dtype (FP32 for BF16) */
    size_t twiddle_bytes;
    size_t scratch_offset;   /* peak-finder counters */
    size_t scratch_bytes;
    int32_t seg_len;         /* L actually used */
    int32_t valid_per_seg;   /* V = L - M */
    int32_t z_chunk;         /* templates per workgroup actually used */
    int32_t bank_elem_bytes; /* bytes per complex template value */
    int32_t algo;            /* kernel family actually used (FDAS_ALGO_VALU or FDAS_ALGO_MFMA) */
    size_t tables_offset;    /* matrix-core operator and twiddle tables (MFMA only) */
    size_t tables_bytes;
} fdas_layout;

/* Create a plan (host only, no device work).  The plan fixes what the
 * search correlates with: the bank of acceleration templates the astronomer
 * chooses (z grid and taps, Section "Detailed explanation": the templates
 * are chosen per search and made once, Section "Template conversion"), the
 * overlap-save segment length and the precision form (Section "Updating the
 * pipeline to bfloat16").  Validates the configuration:
 * FDAS_E_INVALID for n_z < 1, odd or < 2 M, L not a power of two or not in
 * [1024, 16384], M >= L, max_bins < 1, z_step <= 0 with n_z > 1, a plane
 * dtype the compute dtype cannot produce; FDAS_E_UNSUPPORTED for FP8 and for
 * FP64 compute with L > 8192.  On success *out owns a new plan and
 * *workspace_bytes is the device workspace the caller must provide. */
int fdas_plan(const fdas_config *cfg, fdas_plan_t *out, size_t *workspace_bytes);

/* Free a plan (host only).  NULL is ignored. */
void fdas_destroy(fdas_plan_t plan);

/* Attach caller-owned device memory of at least the plan's workspace size
 * (FDAS_E_WORKSPACE if smaller).  Replacing it invalidates the templates. */
int fdas_set_workspace(fdas_plan_t plan, void *dev, size_t bytes);

/* Byte layout of the workspace (host only). */
int fdas_get_layout(fdas_plan_t plan, fdas_layout *out);

/* Build the template bank (Section "Template conversion": templates are made
 * in a higher precision and converted to the reduced one).  In double
 * precision on the GPU: the response through Fresnel integrals, the M taps,
 * their l2 normalisation, the length-L DFT of the circularly placed taps
 * (h[m mod L] = g[m]) scaled by 1/L, then one round-to-nearest-even cast to
 * the compute dtype.  Also writes the twiddle table.  Asynchronous on
 * stream; FDAS_E_WORKSPACE without a workspace. */
int fdas_make_templates(fdas_plan_t plan, void *stream);

/* Spectrum preparation upstream of fdas_correlate (no plan needed): the
 * normalised spectrum of a real time series, with the real FFT in single
 * precision as the paper keeps it (Section "Casting between single-precision
 * and bfloat16"):
 *   X[k] = sum_t x[t] exp(-2 pi i k t / N_t),  k in [0, N_t / 2)  (Nyquist dropped),
 *   X[0] = 0,   X[k] /= sqrt(median_{k >= 1} |X[k]|^2 / ln 2)
 * so that white-noise powers become Exp(1).  The complex FFT of the N_t / 2
 * points z[m] = x[2m] + i x[2m+1] runs as a four-step transform of two passes
 * whose sub-transforms stay in LDS (N_t / 2 = N1 N2 with N1 <= 4096 and
 * N2 <= 2048), the real split fused into the second; other power-of-two
 * lengths take Stockham passes over global memory.  The median is an exact
 * selection.
 *   series     device, n_t floats (8-byte aligned)
 *   n_t        a power of two in [4, 2^28], or 3 * 2^a in [384, 3 * 2^22]
 *              (FDAS_E_UNSUPPORTED otherwise; FDAS_E_INVALID below 4)
 *   spectrum   device, n_t / 2 complex64 (16-byte aligned): the result
 *   workspace  device, at least fdas_prepare_workspace's bytes (16-byte
 *              aligned), FDAS_E_WORKSPACE otherwise
 * Asynchronous on stream; records kernels only (graph-capturable).  An
 * all-zero series has median 0 and gives non-finite values. */
int fdas_prepare_workspace(int64_t n_t, size_t *workspace_bytes);
int fdas_prepare(const float *series, int64_t n_t, void *spectrum, void *workspace, size_t workspace_bytes,
                 void *stream);

/* Template bank of one plane of a jerk search: the same z grid, the taps
 * of a sinusoid whose drift itself changes by w bins over the observation
 * (frequency r0 + z u + w u^2 / 2, u in [0, 1)):
 *   A(q, z, w) = int_0^1 exp(i pi (2 q u + z u^2 + w u^3 / 3)) du,
 *   g_j[m] = conj(A(m - z_j/2 - w/6, z_j, w)) / ||.||_2
 * (r stays the mean frequency).  The paper studies the z search only and
 * describes the jerk search as the same template correlation over an
 * f-fdot-fddot volume (Section "FDAS vs Jerk Search"): one plane per w.
 * The response has no closed form and is integrated on the GPU by composite
 * 16-point Gauss-Legendre quadrature in double precision (panels of at most
 * half a turn of phase); w = 0 is
 * exactly fdas_make_templates (closed form).  The rest as
 * fdas_make_templates: asynchronous on stream, FDAS_E_WORKSPACE without a
 * workspace, FDAS_E_INVALID for a non-finite w; fdas_correlate then writes
 * the plane of this w. */
int fdas_make_templates_jerk(fdas_plan_t plan, double w, void *stream);

/* The f-fdot plane of one spectrum (Section "Detailed explanation": the
 * normalised spectrum correlated with every template by overlap-save --
 * segment transform, product with each template's transform, inverse
 * transform, |.|^2, the contaminated edges of each segment discarded).
 *   spectrum  device, n_bins complex64 values (interleaved re, im floats)
 *   n_bins    N, 1 <= N <= max_bins
 *   plane     device, n_z x N row-major cells of the plan's plane dtype
 * Every cell of the plane is written.  Any N is served; with the L = 4096
 * matrix-core kernel a plane whose rows all start on 16-byte boundaries (N
 * and M / 2 multiples of 8 for BF16, of 4 for FP32) is written fastest,
 * other lengths through 16-byte stores of runs shifted to each row's
 * alignment.
 * FDAS_E_STATE before fdas_make_templates, FDAS_E_INVALID for bad pointers
 * or sizes. */
int fdas_correlate(fdas_plan_t plan, const void *spectrum, int64_t n_bins,
                   void *plane, void *stream);

/* Many spectra of uneven length, e.g. dedispersion trials, correlated with
 * the same template bank in one launch.
 *
 * fdas_set_batch (host, synchronous on stream; call it outside any graph
 * capture) validates the jobs against the caller's buffer sizes (n_bins in
 * [1, max_bins], spec_off + n_bins <= spectra_bins, plane_off + n_z * n_bins
 * <= plane_cells, no negative offsets, n_jobs in [1, max_jobs]) and stores the
 * job table in the workspace.  FDAS_E_INVALID names a bad job; the previous
 * batch is then cleared.
 *
 * fdas_correlate_batch enqueues the batch on stream: a counter reset kernel
 * and one persistent launch whose workgroups pull (job, segment, template
 * chunk) tiles until none is left, each workgroup starting on the template
 * chunk of its XCD so that an XCD's L2 holds only part of the bank (BF16
 * matrix-core plans with L = 4096), or one correlation launch per job (other
 * plans).  It records only kernels, so it
 * can be captured in a HIP graph and replayed; each job's plane is exactly
 * what fdas_correlate writes for that spectrum.  FDAS_E_STATE without
 * templates or a batch. */
int fdas_set_batch(fdas_plan_t plan, const fdas_job *jobs, int32_t n_jobs, int64_t spectra_bins,
                   int64_t plane_cells, void *stream);
int fdas_correlate_batch(fdas_plan_t plan, const void *spectra, void *planes, void *stream);

/* Measured choice of the kernel knobs (segment length, kernel family,
 * templates per workgroup) for a workload: the batched mode serves spectra of
 * several length classes, and the fastest segment length and template chunk
 * depend on the length and the template count.  Synchronous on stream.
 *
 * cfg fixes the workload (max_bins, z grid, taps, compute, plane dtype); each
 * of seg_len, algo and z_chunk that is 0 / FDAS_ALGO_AUTO is searched, a
 * non-zero value is kept.  Candidates: every supported L in [1024, 16384]
 * with L > M (BF16 also on the matrix-core kernels where they exist) and
 * template chunks n_z, ceil(n_z/2), ceil(n_z/4), ceil(n_z/8).  Each one gets
 * a plan on the caller's workspace, its template bank, one warm-up and reps
 * timed fdas_correlate launches on spectrum (n_bins bins) into plane (n_z x
 * n_bins of the plane dtype), timed with HIP events.
 *
 * fdas_tune_workspace gives the workspace size that covers every candidate.
 * fdas_tune writes the fastest configuration (all knobs explicit) to *best
 * and its mean launch time in milliseconds to *best_ms; the workspace content
 * is overwritten (a plan that used it must call fdas_make_templates again).
 * FDAS_E_WORKSPACE if workspace_bytes is below fdas_tune_workspace's value,
 * FDAS_E_UNSUPPORTED if no candidate is valid, FDAS_E_INVALID for bad
 * arguments (reps in [1, 1000]). */
int fdas_tune_workspace(const fdas_config *cfg, size_t *workspace_bytes);
int fdas_tune(const fdas_config *cfg, const void *spectrum, int64_t n_bins, void *plane, void *workspace,
              size_t workspace_bytes, int32_t reps, fdas_config *best, float *best_ms, void *stream);

/* Thresholded peaks of a plane written by fdas_correlate with the same plan
 * (Sections "Detailed explanation" and "Peakfinding methodology").  A cell is
 * a peak iff P > threshold, P > every existing 8-neighbour that precedes it
 * in row-major (z_idx, r) order and P >= every existing 8-neighbour that
 * follows it (edge cells compare only neighbours that exist; NaN is never a
 * peak).  Peaks are written to out (device, capacity entries) in (z_idx, r)
 * order with job = 0; the true count goes to *n_found (device int64).  When
 * the count exceeds capacity the first capacity peaks are written; the call
 * itself cannot know without a device synchronisation and returns FDAS_OK,
 * and fdas_peaks_check then returns FDAS_E_CAPACITY.  The plane
 * pointer needs only the alignment of its element type (a job's plane inside
 * a batch buffer may start anywhere); out 16-byte, n_found 8-byte aligned. */
int fdas_peaks(fdas_plan_t plan, const void *plane, int64_t n_bins, float threshold,
               fdas_peak *out, int64_t capacity, int64_t *n_found, void *stream);

/* Overflow check of peak lists (synchronous; the one call here that waits
 * for the device).  The peak calls cannot see an overflow without a device
 * synchronisation, so they return FDAS_OK and leave the first capacity
 * entries and the true count; this call waits for the work enqueued on
 * stream, copies the n_lists true counts from n_found (device, 8-byte
 * aligned int64) to counts (host, n_lists int64) and returns FDAS_E_CAPACITY
 * when a count exceeds capacity (the lists then hold their first capacity
 * peaks), FDAS_OK otherwise, FDAS_E_INVALID for null pointers, n_lists < 1
 * or capacity < 0.  The Python binding makes this check after every peak
 * call and raises on FDAS_E_CAPACITY unless truncation is asked for. */
int fdas_peaks_check(const int64_t *n_found, int32_t n_lists, int64_t capacity, int64_t *counts, void *stream);

/* Plane and peaks of one spectrum in one call: the plane fdas_correlate
 * writes and exactly the list and count fdas_peaks then gives for it (same
 * arguments, alignment and error rules as the two calls; spectrum and plane
 * 16-byte aligned).  With a BF16 matrix-core plan of L = 4096 the correlation
 * kernel flags the peak finder's tiles (one row x 1024 bins) that hold a
 * stored cell above the threshold while it writes the plane, so the finder
 * reads the plane only around those tiles instead of streaming all of it
 * (peak finding fused into the plane store); other plans run fdas_correlate
 * then fdas_peaks.  Asynchronous on stream, kernels only. */
int fdas_correlate_peaks(fdas_plan_t plan, const void *spectrum, int64_t n_bins, void *plane, float threshold,
                         fdas_peak *out, int64_t capacity, int64_t *n_found, void *stream);

/* Batched form over the batch set by fdas_set_batch: every job's plane, as
 * fdas_correlate_batch writes it, and the peaks of every job's plane.  Job
 * i's list goes to out + i * capacity (capacity entries each, job = i; the
 * list fdas_peaks gives for that plane otherwise) and its true count to
 * n_found[i] (device, n_jobs int64, 8-byte aligned).  The tiles of all jobs'
 * planes share one index space, so one count, one scan and one write launch
 * serve the whole batch; with a BF16 matrix-core plan of L = 4096 the tiles
 * are flagged by the persistent correlation launch itself, other plans add
 * one flagging pass per job.
 *   scratch  caller device memory, 16-byte aligned, at least the bytes
 *            fdas_batch_peaks_workspace gives for the current batch (flags,
 *            counts and offsets: about 6 bytes per 1024 plane cells)
 * fdas_batch_peaks_workspace: FDAS_E_STATE without a batch.
 * fdas_correlate_batch_peaks: asynchronous on stream, kernels only
 * (graph-capturable); FDAS_E_WORKSPACE for a missing or short scratch,
 * FDAS_E_STATE without templates or a batch. */
int fdas_batch_peaks_workspace(fdas_plan_t plan, size_t *scratch_bytes);
int fdas_correlate_batch_peaks(fdas_plan_t plan, const void *spectra, void *planes, float threshold,
                               fdas_peak *out, int64_t capacity, int64_t *n_found, void *scratch,
                               size_t scratch_bytes, void *stream);

/* Band maxima of a plane written by fdas_correlate with the same plan: the
 * paper's own peak finding takes the highest point of each harmonic band
 * (Section "Peakfinding methodology", band bounds in Table 3), and the same
 * reduction over noise-only planes measures the noise canopy (Section
 * "Extreme bin drifts").
 *   windows  device, n_windows x 4 int64 (z_lo, z_hi, r_lo, r_hi): template
 *            rows [z_lo, z_hi) x bins [r_lo, r_hi), clipped to the plane
 *            (8-byte aligned)
 *   out      device, n_windows entries (16-byte aligned): r, z_idx and power
 *            (the plane value as single precision) of the window's highest
 *            cell, job = 0; NaN cells are skipped, ties go to the first cell
 *            in (z_idx, r) order; a window with no non-NaN cell gives
 *            r = z_idx = -1 and power NaN
 * Deterministic (order-independent reductions).  Needs no workspace; out is
 * also the accumulator while the call runs.  FDAS_E_INVALID for bad
 * pointers, n_bins outside [1, max_bins] or n_windows outside [1, 65535]. */
int fdas_band_max(fdas_plan_t plan, const void *plane, int64_t n_bins, const int64_t *windows,
                  int32_t n_windows, fdas_peak *out, void *stream);

/* Incoherent harmonic sum of a plane written by fdas_correlate with the same
 * plan.  Harmonic h of a periodic signal at (r, z) lies at (h r, h z)
 * (Section "Detailed explanation"); the sum gathers the powers of the first
 * n_harm harmonics onto the fundamental's cell:
 *   S[j, r] = sum_{h=1..n_harm} P[j_h, h r],  r in [0, N_H),  N_H = (n_bins - 1) / n_harm + 1,
 *   j_h = floor((h z_j - z_min) / z_step + 1/2)   (nearest template row of h z_j,
 *         a tie going to the upper row; each step one IEEE double operation
 *         in this order, z_j = z_min + j z_step),
 * a term whose row j_h lies outside [0, n_z) being left out (one template:
 * its row is kept for every h when z_min = 0, only for h = 1 otherwise).
 *   plane    device, n_z x n_bins of the plan's plane dtype (element alignment)
 *   n_harm   H, 1..32
 *   out      device, n_z x N_H cells of the plan's plane dtype, row stride N_H
 *            (element alignment); sums in single precision (double for an
 *            FP64 plane), bfloat16 output rounded to nearest even.  fdas_peaks
 *            on out with n_bins = N_H thresholds the summed plane.
 * Needs no workspace.  FDAS_E_INVALID for bad pointers or sizes,
 * FDAS_E_UNSUPPORTED for more than 65535 templates or a plane row of 4 GB
 * less 1 MB or more (n_bins x the plane value size; the same limit holds
 * for every harmonic-sum call below). */
int fdas_harmonic_sum(fdas_plan_t plan, const void *plane, int64_t n_bins, int32_t n_harm, void *out,
                      void *stream);

/* Several harmonic sums in one pass over the plane: for an increasing list
 * n_harm[0] < n_harm[1] < ... (n_levels in [1, 8], each in [1, 32]) the
 * sums fdas_harmonic_sum gives for each, sum l written to outs[l] (device,
 * n_z x ((n_bins - 1) / n_harm[l] + 1) of the plane dtype, element
 * alignment; outs is a host array).  The harmonics are accumulated once in
 * the order h = 1, 2, ..., so each sum is bitwise fdas_harmonic_sum's and
 * the lower harmonics are read once for all sums.  Asynchronous on stream;
 * FDAS_E_INVALID for bad lists or pointers. */
int fdas_harmonic_sums(fdas_plan_t plan, const void *plane, int64_t n_bins, int32_t n_levels,
                       const int32_t *n_harm, void *const *outs, void *stream);

/* The same sums with the thresholded peaks of each: sum l's list (the one
 * fdas_peaks gives for outs[l] with thresholds[l]) goes to peaks[l] (host
 * array of device pointers, capacity entries each, 16-byte aligned), its
 * true count to n_found[l] (device, n_levels int64, 8-byte aligned).  The
 * summing kernel flags the peak tiles of every sum while it stores them, so
 * no sum is streamed back.
 *   scratch  caller device memory (16-byte aligned) of at least the bytes
 *            fdas_harmonic_sums_peaks_workspace gives for the same n_bins
 *            and list: the flags of every sum and the peak counters
 * FDAS_E_UNSUPPORTED for sums of 2^31 bins or tiles and more,
 * FDAS_E_WORKSPACE for a missing or short scratch.  Asynchronous on stream,
 * kernels only. */
int fdas_harmonic_sums_peaks_workspace(fdas_plan_t plan, int64_t n_bins, int32_t n_levels,
                                       const int32_t *n_harm, size_t *scratch_bytes);
int fdas_harmonic_sums_peaks(fdas_plan_t plan, const void *plane, int64_t n_bins, int32_t n_levels,
                             const int32_t *n_harm, void *const *outs, const float *thresholds,
                             fdas_peak *const *peaks, int64_t capacity, int64_t *n_found, void *scratch,
                             size_t scratch_bytes, void *stream);

/* fdas_harmonic_sums_peaks for callers that cannot allocate device memory
 * (code recorded into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc): the same sums, lists and counts, with the scratch taken
 * from a fixed array the library holds on each GPU it runs on until the
 * process ends, FDAS_NOALLOC_SCRATCH_BYTES in size.  The call allocates
 * nothing and calls no allocating routine; the caller still owns the plane,
 * the sums, the peak lists and n_found (arguments and rules as for
 * fdas_harmonic_sums_peaks).  FDAS_E_WORKSPACE when the scratch
 * fdas_harmonic_sums_peaks_workspace gives for these arguments exceeds
 * FDAS_NOALLOC_SCRATCH_BYTES (about 1.7 MB for the sums H = 2, 4, 8, 16 of a
 * 101 x 4,194,304 plane; planes up to about 2.6e9 cells fit at these
 * levels); FDAS_E_HIP if the array's device address cannot be obtained
 * (first call on a device).  Every call on one GPU shares that GPU's array
 * and each call clears the parts it needs on its stream; calls that overlap
 * on one GPU (two streams, or two host threads) race and must be ordered by
 * the caller.  Asynchronous on stream, kernels only. */
#define FDAS_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
int fdas_harmonic_sums_peaks_noalloc(fdas_plan_t plan, const void *plane, int64_t n_bins, int32_t n_levels,
                                     const int32_t *n_harm, void *const *outs, const float *thresholds,
                                     fdas_peak *const *peaks, int64_t capacity, int64_t *n_found, void *stream);

/* The thresholded peaks of several harmonic sums of one plane, the sums
 * never stored (Section "Detailed explanation": the harmonics of a signal at
 * (r, z) sit at (h r, h z)): for each level l exactly the list and true count
 * fdas_harmonic_sums_peaks gives for n_harm[l] and thresholds[l], without
 * writing the n_z x N_H sums.  One summing launch flags the tiles (one row x
 * 1024 fundamentals) where a sum, rounded to the plane's type as a store
 * would round it, may exceed its level's threshold; the finder recomputes the
 * sums of the flagged tiles and their neighbours from the plane in the same
 * order and precision, so every listed cell and power is bitwise the stored
 * sum's.  For a search that only wants the candidates this skips writing
 * (and the finder's reading) the sums.
 *   plane      device, n_z x n_bins of the plane dtype (element alignment)
 *   n_harm, thresholds  host arrays of n_levels (1..8) entries, n_harm
 *              increasing, each in 1..32
 *   peaks      device, n_levels x capacity records (16-byte aligned): level
 *              l's list at peaks + l capacity, job = 0
 *   n_found    device, n_levels int64 (8-byte aligned): true counts
 *   scratch    caller device memory (16-byte aligned) of at least the bytes
 *              fdas_harmonic_peaks_workspace gives for the same n_bins and
 *              levels (a one-job table, flags, counters, list layout,
 *              harmonic rows)
 * Needs no plan workspace or batch.  FDAS_E_INVALID for bad lists, sizes or
 * pointers, FDAS_E_UNSUPPORTED for more than 65535 templates, plane rows of
 * 4 GB less 1 MB or more, or 2^31 tiles or summing workgroups,
 * FDAS_E_WORKSPACE for a missing or short scratch.  Asynchronous on stream,
 * kernels only (graph-capturable): six launches per call. */
int fdas_harmonic_peaks_workspace(fdas_plan_t plan, int64_t n_bins, int32_t n_levels, const int32_t *n_harm,
                                  size_t *scratch_bytes);
int fdas_harmonic_peaks(fdas_plan_t plan, const void *plane, int64_t n_bins, int32_t n_levels, const int32_t *n_harm,
                        const float *thresholds, fdas_peak *peaks, int64_t capacity, int64_t *n_found, void *scratch,
                        size_t scratch_bytes, void *stream);

/* Harmonic summing with thresholding in one call: the summed plane
 * fdas_harmonic_sum writes to out, and exactly the list and count fdas_peaks
 * then gives for it (an n_z x N_H plane, N_H = (n_bins - 1) / n_harm + 1;
 * peaks, capacity and n_found as for fdas_peaks: peaks 16-byte and n_found
 * 8-byte aligned, job = 0).  The summing kernel flags the peak finder's tiles
 * (one row x 1024 bins) holding a stored sum above the threshold while it
 * writes them, so the finder does not stream the summed plane back.  Same
 * argument rules as fdas_harmonic_sum; FDAS_E_WORKSPACE without a workspace
 * (the peak finder's counters live there).  Asynchronous on stream. */
int fdas_harmonic_sum_peaks(fdas_plan_t plan, const void *plane, int64_t n_bins, int32_t n_harm, void *out,
                            float threshold, fdas_peak *peaks, int64_t capacity, int64_t *n_found,
                            void *stream);

/* Harmonic sums with their thresholded peaks for every job of the batch set
 * by fdas_set_batch, in one launch sequence (Section "Detailed explanation":
 * the harmonics of a signal at (r, z) sit at (h r, h z)): for each level l
 * and job i, the peaks fdas_harmonic_sums_peaks lists for job i's plane
 * (at planes + its plane offset, as fdas_correlate_batch writes it) with
 * n_harm[l] and thresholds[l].  The sums themselves are never stored: one
 * summing launch over all jobs flags the tiles (one row x 1024 fundamentals)
 * where a sum, rounded to the plane's type as a store would round it, may
 * exceed its level's threshold, and the finder recomputes the sums of the
 * flagged tiles and their neighbours from the planes, so every listed cell
 * and power is bitwise the stored sum's.
 *   n_harm, thresholds  host arrays of n_levels (1..8) entries, n_harm
 *              increasing, each in 1..32
 *   peaks      device, n_levels x n_jobs x capacity records (16-byte
 *              aligned): list (l, i) at peaks + (l n_jobs + i) capacity, job = i
 *   n_found    device, n_levels x n_jobs int64 (8-byte aligned): true counts
 *   scratch    caller device memory (16-byte aligned) of at least the bytes
 *              fdas_batch_harmonic_sums_peaks_workspace gives for the same
 *              batch and levels (flags, counts, list layout, harmonic rows)
 * FDAS_E_STATE without a batch, FDAS_E_UNSUPPORTED for more than 65535
 * templates or 2^31 tiles or summing workgroups, FDAS_E_WORKSPACE for a
 * missing or short scratch.  Asynchronous on stream, kernels only
 * (graph-capturable): five launches per call. */
int fdas_batch_harmonic_sums_peaks_workspace(fdas_plan_t plan, int32_t n_levels, const int32_t *n_harm,
                                             size_t *scratch_bytes);
int fdas_batch_harmonic_sums_peaks(fdas_plan_t plan, const void *planes, int32_t n_levels, const int32_t *n_harm,
                                   const float *thresholds, fdas_peak *peaks, int64_t capacity, int64_t *n_found,
                                   void *scratch, size_t scratch_bytes, void *stream);

/* Candidate refinement: matched-filter power at continuous (r, z) and its
 * gradient (no plan needed).  The plane samples the power on integer r and a
 * z grid, and quantisation in both axes moves peaks into adjacent bins
 * (Section "Peakfinding methodology"); this evaluates the same matched filter
 * off the grid from the taps spectral bins around r:
 *   F(r, z) = sum_{k = floor(r) - taps/2 + 1}^{floor(r) + taps/2} X[k] conj(A(r - z/2 - k, z)),
 *   P = |F|^2,  dP/dr, dP/dz analytic (X = 0 outside [0, N)).
 *   spectrum   device, n_bins complex64
 *   r, z       device, n_cand doubles each: start points in, final points out
 *   power, dp_dr, dp_dz   device, n_cand doubles each (may be NULL): values at
 *              the final points
 *   taps       even, 2..64 (32 is the usual choice)
 *   n_steps    0: evaluate only; > 0: that many ascent steps
 *              r += eta_r_scale * 3 / (2 pi^2 P) dP/dr,
 *              z += eta_z_scale * 90 / (pi^2 P) dP/dz  (a Newton step on the
 *              curvature of an isolated peak), then evaluate.
 * Positions and arithmetic are FP64 (an FP32 bin index near 4e6 has a
 * spacing of half a bin).  FDAS_E_INVALID for bad sizes or pointers
 * (device pointers 8-byte aligned, the spectrum 8-byte aligned). */
int fdas_refine(const void *spectrum, int64_t n_bins, int32_t n_cand, double *r, double *z,
                double *power, double *dp_dr, double *dp_dz, int32_t taps, int32_t n_steps,
                double eta_r_scale, double eta_z_scale, void *stream);

/* Backward pass of P(r, z) for automatic differentiation: with grad_power
 * the upstream gradient dL/dP, writes grad_r = grad_power * dP/dr and
 * grad_z = grad_power * dP/dz at the given points (all device, n_cand
 * doubles). */
int fdas_refine_backward(const void *spectrum, int64_t n_bins, int32_t n_cand, const double *r,
                         const double *z, const double *grad_power, double *grad_r, double *grad_z,
                         int32_t taps, void *stream);

/* Text for a status code (static storage). */
const char *fdas_strerror(int status);

/* The HIP error code behind the last FDAS_E_HIP on this thread. */
int fdas_last_hip_error(void);

/* Library version, e.g. "0.1.0". */
const char *fdas_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDAS_H */
