// Incoherent harmonic summing over the f-fdot plane.
//
// Harmonic h of a periodic signal at (r, z) sits at (h r, h z) (Section
// "Detailed explanation"), so summing the powers of the first H harmonics
// onto the fundamental's cell gathers a pulsar's power spread over its
// harmonics into one cell:
//   S_H[j, r] = sum_{h=1..H} P[j_h, h r],  r < N_H = floor((N - 1) / H) + 1,
//   j_h = floor((h z_j - z_min) / z_step + 1/2), z_j = z_min + j z_step,
// terms with j_h outside the grid left out (one template: row 0 kept when
// h z_0 = z_0).  The row of each harmonic is a decision taken in double
// precision from the z grid; each step is one IEEE double operation in the
// order written (no fused multiply-add), so the rows are exactly those of
// that definition.
//
// One workgroup per (template row, block of 2048 fundamentals), 8 per thread
// 256 apart; the workgroup's harmonic rows are computed once into LDS.
// Harmonic h of consecutive fundamentals is h bins apart, so the reads of
// harmonic h touch every cache line of an h-times wider span; for a single H
// the cells one row skips are read by other rows' harmonics while the L2
// still holds the lines, and each plane byte comes into L2 about once (the
// several-H pass, whose low harmonics reach further, about 2.5 times).  Sums
// in FP32 (FP64 for an FP64 plane); the output has the plane's dtype
// (bfloat16 rounded to nearest even), so fdas_peaks thresholds it directly.
// The marking form (kMark) also flags the peak finder's tiles of the summed
// plane while storing it, so harmonic summing with thresholding needs no
// second read of the sums.  The batch form (k_batch_sums_mark) sums every
// job of a batch and only flags the tiles; the sums are recomputed for the
// flagged tiles by the peak finder and never stored.
#include "harmonic_rows.hpp"
#include "internal.hpp"

#include <algorithm>
#include <climits>
#include "marks.hpp"
#include "plane_io.hpp"

namespace fdas {

namespace {

constexpr int kHsThreads = 256;
// word 3 of a raw buffer resource on gfx9-family parts (32-bit data format,
// no swizzle; out-of-range offsets read zero)
constexpr int kBufferWord3 = 0x00020000;
constexpr int kHsPerThread = 8;

// plane element -> accumulation type
template <class PT>
struct hs_io;
template <>
struct hs_io<float> {
    using acc = float;
    static __device__ __forceinline__ float get(const float *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ float getb(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
    static __device__ __forceinline__ void put(float *p, float v) { plane_store<float>::put(p, v); }
    // a bound b with: stored value > thr implies v > b (exact here)
    static __device__ __forceinline__ float mark_bound(float thr) { return thr; }
};
template <>
struct hs_io<double> {
    using acc = double;
    static __device__ __forceinline__ double get(const double *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ double getb(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    }
    static __device__ __forceinline__ void put(double *p, double v) { plane_store<double>::put(p, v); }
    static __device__ __forceinline__ double mark_bound(float thr) { return (double)thr; }
};
template <>
struct hs_io<__bf16> {
    using acc = float;
    static __device__ __forceinline__ float get(const __bf16 *p, int64_t i) {
        return __uint_as_float((uint32_t)reinterpret_cast<const unsigned short *>(p)[i] << 16);   // exact
    }
    static __device__ __forceinline__ float getb(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
        return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0) << 16);
    }
    static __device__ __forceinline__ void put(__bf16 *p, float v) { plane_store<__bf16>::put(p, v); }
    // Rounding to nearest bfloat16 moves a normal value by at most 2^-8 of
    // itself, so a stored value above thr > 0 comes from v > thr (1 - 2^-8)
    // (the product's own rounding is far inside that margin); tiny, zero,
    // negative or NaN thresholds pass every value (flags may be a superset).
    static __device__ __forceinline__ float mark_bound(float thr) {
        return thr > 1e-30f ? thr * 0.99609375f : -INFINITY;
    }
};

// Add harmonics h_lo .. h_hi, in that order, of this thread's fundamentals
// r0 + 256 i below lim to acc; rows[h - 1] is harmonic h's row (the same for
// the whole workgroup, -1: left out).  No load sits behind a branch (a
// fundamental or harmonic that is left out reads offset 0 of its row, or a
// zero past the row's end, and keeps its sum), so the kHsPerThread loads of
// a harmonic are in flight together.  A load is a buffer load: the row as a
// buffer resource and the step 256 h i between the thread's fundamentals as
// the scalar offset, so a harmonic costs one 32-bit address register per
// lane (the register file bounds how many loads are in flight on a SIMD).
// A row must hold less than 4 GB (the callers refuse larger rows).
template <class PT>
__device__ __forceinline__ void add_harmonics(typename hs_io<PT>::acc (&acc)[kHsPerThread], const PT *plane,
                                              int64_t n, const int *rows, int h_lo, int h_hi, int64_t r0,
                                              int64_t lim) {
    using A = typename hs_io<PT>::acc;
    const uint32_t ru = (uint32_t)r0;
    const int32_t row_bytes = (int32_t)(uint32_t)(n * (int64_t)sizeof(PT));
    for (int h = h_lo; h <= h_hi; ++h) {
        const int jh = __builtin_amdgcn_readfirstlane(rows[h - 1]);
        const PT *base = plane + (int64_t)max(jh, 0) * n;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<PT *>(base), (short)0, row_bytes, kBufferWord3);
        const uint32_t vo = jh >= 0 ? (uint32_t)h * ru * (uint32_t)sizeof(PT) : 0u;
        const uint32_t step = (uint32_t)h * (uint32_t)(kHsThreads * sizeof(PT));   // uniform
        A v[kHsPerThread];
#pragma unroll
        for (int i = 0; i < kHsPerThread; ++i) v[i] = hs_io<PT>::getb(rs, vo, step * (uint32_t)i);
#pragma unroll
        for (int i = 0; i < kHsPerThread; ++i)
            acc[i] = jh >= 0 && r0 + i * kHsThreads < lim ? acc[i] + v[i] : acc[i];
    }
}

template <class PT, bool kMark>
__global__ void __launch_bounds__(kHsThreads)
k_harmonic_sum(const PT *__restrict__ plane, int64_t n, int n_z, double z_min, double z_step, int n_harm, int64_t nh,
               PT *__restrict__ out, PeakMarks m) {
    using A = typename hs_io<PT>::acc;
    __shared__ int rows[kMaxHarmonics];
    const int j = blockIdx.y;
    if ((int)threadIdx.x < n_harm) rows[threadIdx.x] = harmonic_row(z_min, z_step, n_z, j, threadIdx.x + 1);
    __syncthreads();
    // the workgroup's fundamentals [rb, rb + 2048): thread t takes
    // rb + t + 256 i, so each load instruction of a wave reads one compact run
    // of cache lines and every line is requested once
    const int64_t rb = (int64_t)blockIdx.x * (kHsThreads * kHsPerThread);
    const int64_t r0 = rb + threadIdx.x;
    if (rb >= nh) return;      // uniform: every load below is unconditional
    A acc[kHsPerThread];
#pragma unroll
    for (int i = 0; i < kHsPerThread; ++i) acc[i] = 0;
    // h r <= H (N_H - 1) <= N - 1 for every kept fundamental r < N_H
    add_harmonics<PT>(acc, plane, n, rows, 1, n_harm, r0, nh);
    PT *o = out + (int64_t)j * nh;
#pragma unroll
    for (int i = 0; i < kHsPerThread; ++i) {
        const int64_t r = r0 + i * kHsThreads;
        if (r < nh) hs_io<PT>::put(o + r, acc[i]);
    }
    if constexpr (kMark) {
        // per peak tile (1024 fundamentals) the OR of one compare per kept
        // sum: a NaN sum is never above and cannot hide another sum of the
        // tile (a running maximum would turn NaN at the first NaN)
        constexpr int kPerTile = kPeakTileCols / kHsThreads;
        static_assert(kHsPerThread % kPerTile == 0, "whole tiles per workgroup");
        const A bound = hs_io<PT>::mark_bound(m.thr);
#pragma unroll
        for (int t = 0; t < kHsPerThread / kPerTile; ++t) {
            bool above = false;
#pragma unroll
            for (int i = t * kPerTile; i < (t + 1) * kPerTile; ++i)
                above |= (r0 + i * kHsThreads < nh) & (acc[i] > bound);
            const int64_t rt = rb + (int64_t)t * kPeakTileCols;
            if (above) mark_run(m, (uint32_t)j * (uint32_t)m.n_cb, 0, (int)rt, (int)rt);
        }
    }
}

// Several sums in one pass: S_H for every H of an increasing list, the
// harmonics accumulated once in the order h = 1, 2, ... and each S_H written
// when h reaches H (the same sequence of additions as the single-H kernel,
// so every sum is bitwise the one k_harmonic_sum gives).  A fundamental r
// takes harmonic h only while a requested sum still needs it (r below N_H of
// some H >= h).
constexpr int kMaxSumLevels = 8;

template <class PT>
struct SumLevels {
    int32_t H[kMaxSumLevels];
    int64_t nh[kMaxSumLevels];
    PT *out[kMaxSumLevels];
    PeakMarks marks[kMaxSumLevels];   // marking form: the peak tiles of each sum
};

// kMark: each thread flags, per peak tile of a sum it writes, the tile when
// one of its sums there passes the threshold lowered by the rounding bound
// (flags may be a superset).
template <class PT, bool kMark>
__device__ __forceinline__ void mark_sums(const typename hs_io<PT>::acc (&acc)[kHsPerThread], int64_t r0,
                                          int64_t rb, int64_t lim, int j, const PeakMarks &m) {
    using A = typename hs_io<PT>::acc;
    constexpr int kPerTile = kPeakTileCols / kHsThreads;
    const A bound = hs_io<PT>::mark_bound(m.thr);
#pragma unroll
    for (int t = 0; t < kHsPerThread / kPerTile; ++t) {
        if (rb + (int64_t)t * kPeakTileCols >= lim) break;   // uniform
        bool above = false;   // OR of per-sum compares: a NaN sum hides no other
#pragma unroll
        for (int i = t * kPerTile; i < (t + 1) * kPerTile; ++i)
            above |= (r0 + i * kHsThreads < lim) & (acc[i] > bound);
        const int64_t rt = rb + (int64_t)t * kPeakTileCols;
        if (above) mark_run(m, (uint32_t)j * (uint32_t)m.n_cb, 0, (int)rt, (int)rt);
    }
}

template <class PT, bool kMark>
__global__ void __launch_bounds__(kHsThreads)
k_harmonic_sums(const PT *__restrict__ plane, int64_t n, int n_z, double z_min, double z_step, int n_levels,
                SumLevels<PT> lv) {
    using A = typename hs_io<PT>::acc;
    __shared__ int rows[kMaxHarmonics];
    const int j = blockIdx.y;
    const int h_max = lv.H[n_levels - 1];
    if ((int)threadIdx.x < h_max) rows[threadIdx.x] = harmonic_row(z_min, z_step, n_z, j, threadIdx.x + 1);
    __syncthreads();
    const int64_t rb = (int64_t)blockIdx.x * (kHsThreads * kHsPerThread);
    const int64_t r0 = rb + threadIdx.x;
    if (rb >= lv.nh[0]) return;                 // the largest N_H (smallest H); uniform
    A acc[kHsPerThread];
#pragma unroll
    for (int i = 0; i < kHsPerThread; ++i) acc[i] = 0;
    // level l adds harmonics H_{l-1} + 1 .. H_l to the fundamentals below
    // its N_H (every later sum has an even smaller N_H); the exits are taken
    // by the whole workgroup, threads past N_H are masked
    int h_lo = 1;
    for (int lvl = 0; lvl < n_levels; ++lvl) {
        const int64_t lim = lv.nh[lvl];
        if (rb >= lim) break;
        add_harmonics<PT>(acc, plane, n, rows, h_lo, lv.H[lvl], r0, lim);
        h_lo = lv.H[lvl] + 1;
        PT *o = lv.out[lvl] + (int64_t)j * lim;
#pragma unroll
        for (int i = 0; i < kHsPerThread; ++i) {
            const int64_t r = r0 + i * kHsThreads;
            if (r < lim) hs_io<PT>::put(o + r, acc[i]);
        }
        if constexpr (kMark) mark_sums<PT, kMark>(acc, r0, rb, lim, j, lv.marks[lvl]);
    }
}

// Batch form: the sums of every job of a batch, marking only (the sums are
// never stored).  Workgroup u takes the unit units[u] = (job << 16 | row j,
// block b): fundamentals [2048 b, 2048 b + 2048) of template row j (the
// order of the units is set by k_batch_sums_prep for cache reuse).  At each
// level H_l the sums of this thread are tested against list l * n_jobs +
// job's threshold and its tiles flagged (flags are a superset of the tiles
// holding a stored sum above the threshold, as in the marking form).  rows:
// the [n_z][hmax] harmonic rows, read by scalar loads.
template <class PT>
__global__ void __launch_bounds__(kHsThreads)
k_batch_sums_mark(const PT *__restrict__ planes, const fdas_batch_job *__restrict__ jobs,
                  const SumJob *__restrict__ lists, const int2 *__restrict__ units, int n_jobs, int n_levels,
                  const int32_t *__restrict__ rows, int hmax, uint8_t *flags, uint8_t *cflags) {
    using A = typename hs_io<PT>::acc;
    constexpr int64_t kPerUnit = (int64_t)kHsThreads * kHsPerThread;
    const int2 unit = units[blockIdx.x];
    const int job = unit.x >> 16;
    const int j = unit.x & 0xffff;
    const int64_t rb = (int64_t)unit.y * kPerUnit;
    const int64_t r0 = rb + threadIdx.x;
    const int64_t n = jobs[job].n_bins;
    const PT *plane = planes + jobs[job].plane_off;
    const int32_t *rz = rows + (int64_t)j * hmax;
    A acc[kHsPerThread];
#pragma unroll
    for (int i = 0; i < kHsPerThread; ++i) acc[i] = 0;
    // exits are taken by the whole workgroup; threads past N_H are masked
    int h_lo = 1;
    for (int lvl = 0; lvl < n_levels; ++lvl) {
        const SumJob &sj = lists[lvl * n_jobs + job];
        const int64_t lim = sj.nh;
        if (rb >= lim) break;
        add_harmonics<PT>(acc, plane, n, rz, h_lo, sj.H, r0, lim);
        h_lo = sj.H + 1;
        PeakMarks m;
        m.flags = flags + sj.tile_base;
        m.cflags = cflags + sj.chunk_base;
        m.n_cb = (int32_t)((sj.nh + kPeakTileCols - 1) / kPeakTileCols);
        m.tb = -1;
        m.thr = sj.thr;
        mark_sums<PT, true>(acc, r0, rb, lim, j, m);
    }
}

// Order of the summing workgroups (the unit table).  On a grid whose z_min
// is a multiple of z_step, template j has z_j = m_j z_step and its harmonic
// h lies in the row of m = h m_j, at column h r.  So the templates
// m_j = a m (a = 1, 2, ...), taking fundamentals near a x, all read row q m
// near column q x (q = a h), whatever the split of q into a and h.  Units
// (template j, block b of 2048 fundamentals) of a job are ordered by
// R = floor(b / s_j), s_j = max(|m_j|, 1), then by j, then by b: the units
// of one R read each band of a row between them, so the band comes from
// memory about once instead of once for every harmonic that reads it.  The
// order changes no result; on other grids it is merely an order.  Units of
// job i come after those of the jobs before it.  One wave per (job, R):
// P(R) = sum_j min(s_j R, nb) units come before R, and template j has
// clamp(nb - s_j R, 0, s_j) units in R.
__device__ __forceinline__ int unit_scale(double z_min, double z_step, int j) {
    const int m = (int)rint((z_min + (double)j * z_step) / z_step);
    return m < 0 ? (m == INT_MIN ? INT_MAX : -m) : (m == 0 ? 1 : m);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ void build_units(const fdas_batch_job *__restrict__ jobs, int n_jobs, int H0, int n_z, double z_min,
                            double z_step, int2 *units) {
    constexpr int64_t kPerUnit = (int64_t)kHsThreads * kHsPerThread;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t tb = 0, ub = 0;          // first task (R of job i) and first unit of job i
    for (int i = 0; i < n_jobs; ++i) {
        const int64_t nh = (jobs[i].n_bins - 1) / H0 + 1;
        const int64_t nb = (nh + kPerUnit - 1) / kPerUnit;
        for (int64_t R = ((wave - tb) % n_waves + n_waves) % n_waves; R < nb; R += n_waves) {
            int64_t P = 0;
            for (int j = lane; j < n_z; j += 64) P += min((int64_t)unit_scale(z_min, z_step, j) * R, nb);
            P = wave_sum64(P);
            int64_t carry = 0;
            for (int j0 = 0; j0 < n_z; j0 += 64) {
                const int j = j0 + lane;
                int64_t c = 0, first = 0;
                if (j < n_z) {
                    const int64_t sj = unit_scale(z_min, z_step, j);
                    first = sj * R;
                    c = max((int64_t)0, min(nb - first, sj));
                }
                int64_t incl = c;           // inclusive scan over the wave
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int64_t v = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += v;
                }
                const int64_t pos = ub + P + carry + incl - c;
                for (int64_t k = 0; k < c; ++k) units[pos + k] = make_int2((i << 16) | j, (int)(first + k));
                carry += __shfl(incl, 63, 64);
            }
        }
        tb += nb;
        ub += (int64_t)n_z * nb;
    }
}

// Set-up of a batch sums call (one launch): every workgroup clears its share
// of the flags and per-list totals; workgroup 0 lays out the lists (level
// by level, job by job: columns, first tile, first chunk, and for the first
// level the first summing workgroup) by prefix sums; workgroup 1 computes
// the harmonic rows.
struct SumLevelsArg {
    int32_t H[kMaxSumLevels];
    float thr[kMaxSumLevels];
};

__global__ void __launch_bounds__(1024)
k_batch_sums_prep(const fdas_batch_job *__restrict__ jobs, int n_jobs, int n_levels, SumLevelsArg lv, int n_z,
                  double z_min, double z_step, SumJob *lists, int32_t *rows, int hmax, int2 *units,
                  uint8_t *clear, int64_t clear_bytes) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < clear_bytes;
         i += (int64_t)gridDim.x * blockDim.x)
        clear[i] = 0;
    build_units(jobs, n_jobs, lv.H[0], n_z, z_min, z_step, units);
    if (blockIdx.x == 1) {
        for (int i = threadIdx.x; i < n_z * hmax; i += blockDim.x)
            rows[i] = harmonic_row(z_min, z_step, n_z, i / hmax, i % hmax + 1);
    }
    if (blockIdx.x != 0) return;
    __shared__ int64_t part[3][1024];
    __shared__ int64_t carry[3];
    if (threadIdx.x < 3) carry[threadIdx.x] = 0;
    const int S = n_levels * n_jobs;
    const int64_t per_block = (int64_t)kHsThreads * kHsPerThread;
    for (int s0 = 0; s0 < S; s0 += 1024) {
        const int s = s0 + (int)threadIdx.x;
        int64_t nh = 0, tiles = 0, chunks = 0, blocks = 0;
        if (s < S) {
            const int l = s / n_jobs, i = s - l * n_jobs;
            nh = (jobs[i].n_bins - 1) / lv.H[l] + 1;
            tiles = (int64_t)n_z * ((nh + kPeakTileCols - 1) / kPeakTileCols);
            chunks = (tiles + kPeakTilesPerChunk - 1) / kPeakTilesPerChunk;
            if (l == 0) blocks = (int64_t)n_z * ((nh + per_block - 1) / per_block);
        }
        part[0][threadIdx.x] = tiles;
        part[1][threadIdx.x] = chunks;
        part[2][threadIdx.x] = blocks;
        __syncthreads();
        for (int w = 1; w < 1024; w <<= 1) {
            int64_t v[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) v[q] = threadIdx.x >= (unsigned)w ? part[q][threadIdx.x - w] : 0;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q) part[q][threadIdx.x] += v[q];
            __syncthreads();
        }
        if (s < S) {
            const int l = s / n_jobs, i = s - l * n_jobs;
            SumJob sj;
            sj.nh = nh;
            sj.tile_base = carry[0] + part[0][threadIdx.x] - tiles;
            sj.chunk_base = carry[1] + part[1][threadIdx.x] - chunks;
            sj.block_base = carry[2] + part[2][threadIdx.x] - blocks;
            sj.H = lv.H[l];
            sj.job = i;
            sj.thr = lv.thr[l];
            sj.level = l;
            lists[s] = sj;
        }
        __syncthreads();
        if (threadIdx.x < 3) carry[threadIdx.x] += part[threadIdx.x][1023];
        __syncthreads();
    }
}

template <class PT, bool kMark>
hipError_t run_sums(const fdas_plan_s &p, const void *plane, int64_t n, int n_levels, const int32_t *H,
                    void *const *outs, const PeakMarks *marks, hipStream_t st) {
    SumLevels<PT> lv{};
    for (int l = 0; l < n_levels; ++l) {
        lv.H[l] = H[l];
        lv.nh[l] = (n - 1) / H[l] + 1;
        lv.out[l] = static_cast<PT *>(outs[l]);
        if (marks) lv.marks[l] = marks[l];
    }
    const int64_t per_block = (int64_t)kHsThreads * kHsPerThread;
    const int64_t bx = (lv.nh[0] + per_block - 1) / per_block;
    if (bx > 0x7fffffffLL || p.cfg.n_z > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_harmonic_sums<PT, kMark>), dim3((unsigned)bx, (unsigned)p.cfg.n_z), dim3(kHsThreads), 0, st,
                       static_cast<const PT *>(plane), n, p.cfg.n_z, p.cfg.z_min, p.cfg.z_step, n_levels, lv);
    return hipGetLastError();
}

template <class PT, bool kMark>
hipError_t run(const fdas_plan_s &p, const void *plane, int64_t n, int n_harm, void *out, const PeakMarks &m,
               hipStream_t st) {
    const int64_t nh = (n - 1) / n_harm + 1;
    const int64_t per_block = (int64_t)kHsThreads * kHsPerThread;
    const int64_t bx = (nh + per_block - 1) / per_block;
    if (bx > 0x7fffffffLL || p.cfg.n_z > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_harmonic_sum<PT, kMark>), dim3((unsigned)bx, (unsigned)p.cfg.n_z), dim3(kHsThreads), 0, st,
                       static_cast<const PT *>(plane), n, p.cfg.n_z, p.cfg.z_min, p.cfg.z_step, n_harm, nh,
                       static_cast<PT *>(out), m);
    return hipGetLastError();
}

template <bool kMark>
hipError_t dispatch(const fdas_plan_s &p, const void *plane, int64_t n, int n_harm, void *out, const PeakMarks &m,
                    hipStream_t st) {
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32: return run<float, kMark>(p, plane, n, n_harm, out, m, st);
        case FDAS_BF16: return run<__bf16, kMark>(p, plane, n, n_harm, out, m, st);
        case FDAS_FP64: return run<double, kMark>(p, plane, n, n_harm, out, m, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_harmonic_sum(const fdas_plan_s &p, const void *plane, int64_t n, int n_harm, void *out,
                               hipStream_t st) {
    return dispatch<false>(p, plane, n, n_harm, out, PeakMarks{}, st);
}

hipError_t launch_harmonic_sums(const fdas_plan_s &p, const void *plane, int64_t n, int n_levels, const int32_t *H,
                                void *const *outs, const PeakMarks *marks, hipStream_t st) {
    if (marks) {
        switch (p.cfg.plane_dtype) {
            case FDAS_FP32: return run_sums<float, true>(p, plane, n, n_levels, H, outs, marks, st);
            case FDAS_BF16: return run_sums<__bf16, true>(p, plane, n, n_levels, H, outs, marks, st);
            case FDAS_FP64: return run_sums<double, true>(p, plane, n, n_levels, H, outs, marks, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32: return run_sums<float, false>(p, plane, n, n_levels, H, outs, nullptr, st);
        case FDAS_BF16: return run_sums<__bf16, false>(p, plane, n, n_levels, H, outs, nullptr, st);
        case FDAS_FP64: return run_sums<double, false>(p, plane, n, n_levels, H, outs, nullptr, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_harmonic_sum_marked(const fdas_plan_s &p, const void *plane, int64_t n, int n_harm, void *out,
                                      const PeakMarks &marks, hipStream_t st) {
    return dispatch<true>(p, plane, n, n_harm, out, marks, st);
}

BatchSumsLayout batch_sums_layout(const fdas_plan_s &p, const SumBatch &b, int n_levels, const int32_t *H) {
    BatchSumsLayout L;
    const int64_t J = b.n_jobs, S = (int64_t)n_levels * J;
    const int64_t per_block = (int64_t)kHsThreads * kHsPerThread;
    for (int l = 0; l < n_levels; ++l)
        for (int64_t i = 0; i < J; ++i) {
            const fdas_batch_job &j = b.host[i];
            const int64_t nh = (j.n_bins - 1) / H[l] + 1;
            const int64_t tiles = (int64_t)p.cfg.n_z * ((nh + kPeakTileCols - 1) / kPeakTileCols);
            L.tiles += tiles;
            L.chunks += (tiles + kPeakTilesPerChunk - 1) / kPeakTilesPerChunk;
            if (l == 0) L.blocks += (int64_t)p.cfg.n_z * ((nh + per_block - 1) / per_block);
        }
    L.lists = S;
    L.hmax = H[n_levels - 1];
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    L.off_counts = off;
    off = up(off + (size_t)L.tiles * 4);
    L.off_block_counts = off;
    off = up(off + (size_t)L.chunks * 4);
    L.off_wg_totals = off;
    off = up(off + (size_t)kPeakRanges * 4);
    L.off_wg_offsets = off;
    off = up(off + (size_t)(kPeakRanges + 1) * 8);
    L.off_prefix = off;
    off = up(off + (size_t)S * 8);
    L.off_totals = off;                        // per-list totals, then tile flags, then chunk flags
    L.clear_bytes = (size_t)S * 8 + (size_t)L.tiles + (size_t)L.chunks;
    off = up(off + L.clear_bytes);
    L.off_lists = off;
    off = up(off + (size_t)S * sizeof(SumJob));
    L.off_rows = off;
    off = up(off + (size_t)p.cfg.n_z * L.hmax * 4);
    L.off_units = off;
    off = up(off + (size_t)L.blocks * 8);
    L.bytes = off;
    return L;
}

namespace {
__global__ void k_one_job(fdas_batch_job *dst, int64_t n) { *dst = fdas_batch_job{0, n, 0, 0, 0, 0}; }

template <class PT>
hipError_t run_batch_sums(const fdas_plan_s &p, const SumBatch &b, const BatchSumsLayout &L, const void *planes,
                          int n_levels, const int32_t *H, const float *thr, unsigned char *scratch, hipStream_t st) {
    const fdas_batch_job *jobs = b.dev;
    SumLevelsArg lv{};
    for (int l = 0; l < n_levels; ++l) {
        lv.H[l] = H[l];
        lv.thr[l] = thr[l];
    }
    auto *lists = reinterpret_cast<SumJob *>(scratch + L.off_lists);
    auto *rows = reinterpret_cast<int32_t *>(scratch + L.off_rows);
    uint8_t *clear = scratch + L.off_totals;
    uint8_t *flags = clear + (size_t)L.lists * 8;
    uint8_t *cflags = flags + L.tiles;
    // enough workgroups for the clearing and for the unit table (one wave per (job, R))
    const int64_t tasks = L.blocks / std::max(p.cfg.n_z, 1);
    const unsigned cg = (unsigned)std::max<int64_t>(
        2, std::min<int64_t>(1024, std::max<int64_t>((L.clear_bytes + 4095) / 4096, (tasks + 15) / 16)));
    auto *units = reinterpret_cast<int2 *>(scratch + L.off_units);
    hipLaunchKernelGGL(k_batch_sums_prep, dim3(cg), dim3(1024), 0, st, jobs, b.n_jobs, n_levels, lv, p.cfg.n_z,
                       p.cfg.z_min, p.cfg.z_step, lists, rows, L.hmax, units, clear, (int64_t)L.clear_bytes);
    if (L.blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_batch_sums_mark<PT>), dim3((unsigned)L.blocks), dim3(kHsThreads), 0, st,
                       static_cast<const PT *>(planes), jobs, lists, units, b.n_jobs, n_levels, rows, L.hmax,
                       flags, cflags);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_batch_sums_mark(const fdas_plan_s &p, const SumBatch &b, const BatchSumsLayout &L,
                                  const void *planes, int n_levels, const int32_t *H, const float *thr, void *scratch,
                                  hipStream_t st) {
    auto *sc = static_cast<unsigned char *>(scratch);
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32: return run_batch_sums<float>(p, b, L, planes, n_levels, H, thr, sc, st);
        case FDAS_BF16: return run_batch_sums<__bf16>(p, b, L, planes, n_levels, H, thr, sc, st);
        case FDAS_FP64: return run_batch_sums<double>(p, b, L, planes, n_levels, H, thr, sc, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t write_one_job(fdas_batch_job *dev, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_one_job, dim3(1), dim3(1), 0, st, dev, n);
    return hipGetLastError();
}

}  // namespace fdas
