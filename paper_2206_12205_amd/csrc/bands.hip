// Band maxima: the highest cell of each (z, r) window of a plane.
//
// The paper's own peak finding takes the highest point of each harmonic band
// of the plane (Section "Peakfinding methodology", band bounds in Table 3);
// the same reduction over narrow windows measures the noise canopy (the
// height of the highest noise cell in a band, Section "Extreme bin drifts").
// For window (z_lo, z_hi, r_lo, r_hi), half-open and clipped to the plane:
// the largest value, NaN cells skipped, ties to the first cell in (z_idx, r)
// order.
//
// A grid of (workgroups, windows): each workgroup takes (row, 4096-column
// chunk) items of its window in turn.  The value is ranked by an
// order-preserving unsigned key (a NaN-free total order of the plane type).
// FP32 and BF16 planes of fewer than 2^32 cells take one pass: the 32-bit
// value key above the complement of the cell's row-major position in its
// window, so one 64-bit maximum (one atomicMax per workgroup) finds the
// largest value and its first cell together.  FP64 planes take two passes:
//   max   the largest value key, one atomicMax per workgroup;
//   first the smallest row-major position holding that value, one atomicMin
//         per workgroup.
// All results are order-independent, so the output is deterministic.  The
// 64-bit accumulators of window b live in out[b] itself (the r field and
// the z_idx/job pair) until a final kernel writes the peak record.
#include "internal.hpp"

namespace fdas {

namespace {

constexpr int kBandThreads = 256;
constexpr int kBandChunk = 4096;   // columns per work item
constexpr int kBandGrid = 64;      // workgroups per window

// order-preserving keys (larger value -> larger key), NaN never used
__device__ __forceinline__ uint64_t band_key(float v) {
    const uint32_t u = __float_as_uint(v);
    return (uint64_t)((u & 0x80000000u) ? ~u : (u | 0x80000000u));
}
__device__ __forceinline__ uint64_t band_key(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double band_value(uint64_t k, bool dbl) {
    if (dbl) {
        const uint64_t u = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
        return __longlong_as_double((long long)u);
    }
    const uint32_t k32 = (uint32_t)k;
    const uint32_t u = (k32 & 0x80000000u) ? (k32 & 0x7fffffffu) : ~k32;
    return (double)__uint_as_float(u);
}

template <class PT>
struct band_io;
template <>
struct band_io<float> {
    using V = float;
    static __device__ __forceinline__ float get(const float *p, int64_t i) { return p[i]; }
};
template <>
struct band_io<double> {
    using V = double;
    static __device__ __forceinline__ double get(const double *p, int64_t i) { return p[i]; }
};
template <>
struct band_io<unsigned short> {
    using V = float;
    static __device__ __forceinline__ float get(const unsigned short *p, int64_t i) {
        return __uint_as_float((uint32_t)p[i] << 16);   // exact widening of raw bfloat16
    }
};

struct Win {
    int64_t z_lo, z_hi, r_lo, r_hi, n_items, chunks;
};

__device__ __forceinline__ Win band_window(const int64_t *windows, int b, int n_z, int64_t n) {
    Win w;
    w.z_lo = max(windows[4 * b + 0], (int64_t)0);
    w.z_hi = min(windows[4 * b + 1], (int64_t)n_z);
    w.r_lo = max(windows[4 * b + 2], (int64_t)0);
    w.r_hi = min(windows[4 * b + 3], n);
    if (w.z_hi <= w.z_lo || w.r_hi <= w.r_lo) {
        w.n_items = 0;
        w.chunks = 0;
    } else {
        w.chunks = (w.r_hi - w.r_lo + kBandChunk - 1) / kBandChunk;
        w.n_items = (w.z_hi - w.z_lo) * w.chunks;
    }
    return w;
}

__global__ void k_band_clear(fdas_peak *out, int n_windows) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_windows) return;
    uint64_t *acc = reinterpret_cast<uint64_t *>(&out[b]);
    acc[0] = 0;            // largest key (0: no cell yet)
    acc[1] = ~0ull;        // first position holding it
}

template <class PT, bool kFirst>
__global__ void __launch_bounds__(kBandThreads)
k_band_pass(const PT *plane, int64_t n, int n_z, const int64_t *windows, fdas_peak *out) {
    using V = typename band_io<PT>::V;
    __shared__ uint64_t red[kBandThreads];
    const int b = blockIdx.y;
    const Win w = band_window(windows, b, n_z, n);
    uint64_t *acc = reinterpret_cast<uint64_t *>(&out[b]);
    const uint64_t target = kFirst ? acc[0] : 0;
    uint64_t best = kFirst ? ~0ull : 0;
    for (int64_t it = blockIdx.x; it < w.n_items; it += gridDim.x) {
        const int64_t z = w.z_lo + it / w.chunks;
        const int64_t c0 = w.r_lo + (it % w.chunks) * kBandChunk;
        const int64_t c1 = min(c0 + kBandChunk, w.r_hi);
        const PT *row = plane + z * n;
        for (int64_t c = c0 + threadIdx.x; c < c1; c += kBandThreads) {
            const V v = band_io<PT>::get(row, c);
            if (v != v) continue;                                  // NaN
            const uint64_t k = band_key(v);
            if constexpr (kFirst) {
                if (k == target) best = min(best, (uint64_t)(z * n + c));
            } else {
                best = max(best, k);
            }
        }
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = kBandThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            red[threadIdx.x] = kFirst ? min(red[threadIdx.x], red[threadIdx.x + s])
                                      : max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if constexpr (kFirst) {
            if (red[0] != ~0ull) atomicMin(reinterpret_cast<unsigned long long *>(&acc[1]), red[0]);
        } else {
            if (red[0] != 0) atomicMax(reinterpret_cast<unsigned long long *>(&acc[0]), red[0]);
        }
    }
}

// One pass for 32-bit value keys: (key << 32) | (2^32 - 1 - window position).
template <class PT>
__global__ void __launch_bounds__(kBandThreads)
k_band_pass1(const PT *plane, int64_t n, int n_z, const int64_t *windows, fdas_peak *out) {
    using V = typename band_io<PT>::V;
    static_assert(sizeof(V) == 4, "32-bit value keys");
    __shared__ uint64_t red[kBandThreads];
    const int b = blockIdx.y;
    const Win w = band_window(windows, b, n_z, n);
    uint64_t *acc = reinterpret_cast<uint64_t *>(&out[b]);
    const int64_t width = w.r_hi - w.r_lo;
    uint64_t best = 0;
    for (int64_t it = blockIdx.x; it < w.n_items; it += gridDim.x) {
        const int64_t zr = it / w.chunks;   // row inside the window
        const int64_t c0 = w.r_lo + (it % w.chunks) * kBandChunk;
        const int64_t c1 = min(c0 + kBandChunk, w.r_hi);
        const PT *row = plane + (w.z_lo + zr) * n;
        const uint64_t pos0 = (uint64_t)(zr * width - w.r_lo);
        for (int64_t c = c0 + threadIdx.x; c < c1; c += kBandThreads) {
            const V v = band_io<PT>::get(row, c);
            if (v != v) continue;                                  // NaN
            const uint64_t k = (band_key(v) << 32) | (0xffffffffull - (pos0 + (uint64_t)c));
            best = max(best, k);
        }
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = kBandThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != 0) atomicMax(reinterpret_cast<unsigned long long *>(&acc[0]), red[0]);
}

__global__ void k_band_finish1(fdas_peak *out, int n_windows, const int64_t *windows, int n_z, int64_t n) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_windows) return;
    const uint64_t k = reinterpret_cast<const uint64_t *>(&out[b])[0];
    const Win w = band_window(windows, b, n_z, n);
    fdas_peak pk;
    pk.job = 0;
    pk.reserved = 0.0f;
    if (k == 0) {
        pk.r = -1;
        pk.z_idx = -1;
        pk.power = __int_as_float(0x7fc00000);   // NaN
    } else {
        const int64_t width = w.r_hi - w.r_lo;
        const int64_t pos = (int64_t)(0xffffffffull - (k & 0xffffffffull));
        pk.r = w.r_lo + pos % width;
        pk.z_idx = (int32_t)(w.z_lo + pos / width);
        pk.power = (float)band_value(k >> 32, false);
    }
    out[b] = pk;
}

__global__ void k_band_finish(fdas_peak *out, int n_windows, int64_t n, bool dbl) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_windows) return;
    const uint64_t *acc = reinterpret_cast<const uint64_t *>(&out[b]);
    const uint64_t key = acc[0], pos = acc[1];
    fdas_peak pk;
    pk.job = 0;
    pk.reserved = 0.0f;
    if (key == 0 || pos == ~0ull) {
        pk.r = -1;
        pk.z_idx = -1;
        pk.power = __int_as_float(0x7fc00000);   // NaN
    } else {
        pk.r = (int64_t)(pos % (uint64_t)n);
        pk.z_idx = (int32_t)(pos / (uint64_t)n);
        pk.power = (float)band_value(key, dbl);
    }
    out[b] = pk;
}

template <class PT>
hipError_t run(const fdas_plan_s &p, const PT *plane, int64_t n, const int64_t *windows, int n_windows,
               fdas_peak *out, hipStream_t st) {
    const unsigned gb = (unsigned)((n_windows + 255) / 256);
    const dim3 grid(kBandGrid, (unsigned)n_windows);
    hipLaunchKernelGGL(k_band_clear, dim3(gb), dim3(256), 0, st, out, n_windows);
    if constexpr (sizeof(typename band_io<PT>::V) == 4) {
        if ((int64_t)p.cfg.n_z * n < ((int64_t)1 << 32)) {   // every clipped window position fits 32 bits
            hipLaunchKernelGGL((k_band_pass1<PT>), grid, dim3(kBandThreads), 0, st, plane, n, p.cfg.n_z, windows,
                               out);
            hipLaunchKernelGGL(k_band_finish1, dim3(gb), dim3(256), 0, st, out, n_windows, windows, p.cfg.n_z, n);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_band_pass<PT, false>), grid, dim3(kBandThreads), 0, st, plane, n, p.cfg.n_z, windows, out);
    hipLaunchKernelGGL((k_band_pass<PT, true>), grid, dim3(kBandThreads), 0, st, plane, n, p.cfg.n_z, windows, out);
    hipLaunchKernelGGL(k_band_finish, dim3(gb), dim3(256), 0, st, out, n_windows, n, sizeof(PT) == 8);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_band_max(const fdas_plan_s &p, const void *plane, int64_t n, const int64_t *windows,
                           int32_t n_windows, fdas_peak *out, hipStream_t st) {
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32: return run<float>(p, static_cast<const float *>(plane), n, windows, n_windows, out, st);
        case FDAS_BF16:
            return run<unsigned short>(p, static_cast<const unsigned short *>(plane), n, windows, n_windows, out,
                                       st);
        case FDAS_FP64: return run<double>(p, static_cast<const double *>(plane), n, windows, n_windows, out, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdas
