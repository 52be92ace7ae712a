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
// 256 apart; the workgroup's harmonic rows are computed once
// into LDS.  Harmonic h of consecutive fundamentals is h bins apart, so the
// reads of harmonic h touch every cache line of an h-times wider span: the
// kernel reads about (H + 1) / 2 planes' worth of cache lines, held in part
// by the L2 and the last-level cache.  Sums in FP32 (FP64 for an FP64
// plane); the output has the plane's dtype (bfloat16 rounded to nearest
// even), so fdas_peaks thresholds it directly.  The marking form (kMark)
// also flags the peak finder's tiles of the summed plane while storing it,
// so harmonic summing with thresholding needs no second read of the sums.
#include "internal.hpp"
#include "marks.hpp"
#include "plane_io.hpp"

namespace fdas {

namespace {

constexpr int kHsThreads = 256;
constexpr int kHsPerThread = 8;

__device__ int harmonic_row(double z_min, double z_step, int n_z, int j, int h) {
#pragma clang fp contract(off)
    if (n_z == 1) return ((double)h * z_min == z_min) ? 0 : -1;
    const double t = z_min + (double)j * z_step;
    const double u = (double)h * t;
    const double v = u - z_min;
    const double x = v / z_step;
    const double f = floor(x + 0.5);
    if (!(f >= 0.0 && f < (double)n_z)) return -1;   // outside the grid (or NaN)
    return (int)f;
}

// plane element -> accumulation type
template <class PT>
struct hs_io;
template <>
struct hs_io<float> {
    using acc = float;
    static __device__ __forceinline__ float get(const float *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void put(float *p, float v) { plane_store<float>::put(p, v); }
    // a bound b with: stored value > thr implies v > b (exact here)
    static __device__ __forceinline__ float mark_bound(float thr) { return thr; }
};
template <>
struct hs_io<double> {
    using acc = double;
    static __device__ __forceinline__ double get(const double *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void put(double *p, double v) { plane_store<double>::put(p, v); }
    static __device__ __forceinline__ double mark_bound(float thr) { return (double)thr; }
};
template <>
struct hs_io<__bf16> {
    using acc = float;
    static __device__ __forceinline__ float get(const __bf16 *p, int64_t i) {
        return __uint_as_float((uint32_t)reinterpret_cast<const unsigned short *>(p)[i] << 16);   // exact
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
    if (r0 >= nh) return;
    A acc[kHsPerThread];
#pragma unroll
    for (int i = 0; i < kHsPerThread; ++i) acc[i] = 0;
    // h r <= H (N_H - 1) <= N - 1 for every kept fundamental r < N_H
    for (int h = 1; h <= n_harm; ++h) {
        const int jh = rows[h - 1];
        if (jh < 0) continue;
        const PT *row = plane + (int64_t)jh * n;
#pragma unroll
        for (int i = 0; i < kHsPerThread; ++i) {
            const int64_t r = r0 + i * kHsThreads;
            if (r < nh) acc[i] += hs_io<PT>::get(row, (int64_t)h * r);
        }
    }
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
        if (r0 + t * kPerTile * kHsThreads >= lim) break;
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
    if (r0 >= lv.nh[0]) return;                 // the largest N_H (smallest H)
    A acc[kHsPerThread];
#pragma unroll
    for (int i = 0; i < kHsPerThread; ++i) acc[i] = 0;
    int lvl = 0;
    for (int h = 1; h <= h_max; ++h) {
        const int64_t lim = lv.nh[lvl];         // fundamentals that still need harmonic h
        if (r0 >= lim) break;                   // every later sum has an even smaller N_H
        const int jh = rows[h - 1];
        if (jh >= 0) {
            const PT *row = plane + (int64_t)jh * n;
#pragma unroll
            for (int i = 0; i < kHsPerThread; ++i) {
                const int64_t r = r0 + i * kHsThreads;
                if (r < lim) acc[i] += hs_io<PT>::get(row, (int64_t)h * r);
            }
        }
        if (h == lv.H[lvl]) {
            PT *o = lv.out[lvl] + (int64_t)j * lim;
#pragma unroll
            for (int i = 0; i < kHsPerThread; ++i) {
                const int64_t r = r0 + i * kHsThreads;
                if (r < lim) hs_io<PT>::put(o + r, acc[i]);
            }
            if constexpr (kMark) mark_sums<PT, kMark>(acc, r0, rb, lim, j, lv.marks[lvl]);
            if (++lvl == n_levels) break;
        }
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

}  // namespace fdas
