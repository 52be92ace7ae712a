// Thresholded peak finding on the f-fdot plane.
//
// A pulsar appears as a peak on the plane (Section "Detailed explanation");
// the paper's own analysis picks the highest point of each harmonic band
// (Section "Peakfinding methodology") but does not describe a general peak
// finder.  This one reports every cell that is above the threshold and is a
// 3x3 local maximum: P > thr, P > each existing neighbour that precedes it in
// row-major (z_idx, r) order and P >= each one that follows it.  Comparisons
// are exact (values widened to double), NaN never qualifies.
//
// Deterministic scheme with one tile = one plane row x kPeakTileCols
// columns, tiles numbered in (z_idx, column block) order and grouped in
// chunks of 16 consecutive tiles:
//   mark   one streaming pass flags the tiles (and their chunks) that hold a
//          cell above the threshold;
//   count  every flagged tile counts its peaks; per chunk the total (zero for
//          a chunk without flags);
//   scan   one workgroup turns the per-chunk totals into exclusive offsets
//          and the total;
//   write  every tile with peaks recomputes them and writes them at its offset
//          in column order, dropping those at or beyond the capacity.
// The count and write kernels run a fixed grid that strides over the chunks
// and skips unflagged chunks after one byte read, so a plane with few peaks
// costs one streaming read plus a few thousand workgroups.  The list is
// sorted by (z_idx, r) with no sort pass.
#include <algorithm>
#include <type_traits>

#include "internal.hpp"

namespace fdas {

constexpr int kPeakThreads = 256;
constexpr int kCellsPerThread = kPeakTileCols / kPeakThreads;   // 4

// offsets (int64), totals (int32) and flags (uint8) per chunk of 16 tiles,
// counts (int32) and flags (uint8) per tile
size_t peak_scratch_bytes(int64_t n_tiles) {
    return (size_t)n_tiles * (sizeof(int32_t) + sizeof(int64_t)) + 256;
}

template <class PT>
__device__ __forceinline__ double plane_val(const PT *p, int64_t i);
template <>
__device__ __forceinline__ double plane_val<float>(const float *p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ double plane_val<double>(const double *p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ double plane_val<unsigned short>(const unsigned short *p, int64_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);   // exact widening of raw bfloat16
}

// Stage rows z-1..z+1, columns c0-1 .. c0+kPeakTileCols into LDS (-inf outside
// the plane) and flag this thread's kCellsPerThread consecutive cells.
// Neighbourhood values are compared in the plane's own precision widened to
// float (BF16, FP32: exact) or double (FP64); the threshold is a float.
template <class PT>
using peak_val_t = typename std::conditional<sizeof(PT) == 8, double, float>::type;

template <class PT>
__device__ __forceinline__ int tile_flags(const PT *plane, int64_t n, int n_z, int z, int64_t c0, float thr_f,
                                          peak_val_t<PT> (*buf)[kPeakTileCols + 2], bool *flag) {
    using V = peak_val_t<PT>;
    const V thr = (V)thr_f;
    for (int i = threadIdx.x; i < 3 * (kPeakTileCols + 2); i += kPeakThreads) {
        const int row = i / (kPeakTileCols + 2);
        const int col = i % (kPeakTileCols + 2);
        const int zz = z + row - 1;
        const int64_t cc = c0 + col - 1;
        V v = -INFINITY;
        if (zz >= 0 && zz < n_z && cc >= 0 && cc < n) v = (V)plane_val<PT>(plane, (int64_t)zz * n + cc);
        buf[row][col] = v;
    }
    __syncthreads();
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < kCellsPerThread; ++q) {
        const int col = threadIdx.x * kCellsPerThread + q + 1;
        const int64_t cc = c0 + col - 1;
        const V c = buf[1][col];
        bool ok = cc < n && c > thr;
        // preceding neighbours (strict), following neighbours (non-strict)
        ok = ok && c > buf[0][col - 1] && c > buf[0][col] && c > buf[0][col + 1] && c > buf[1][col - 1];
        ok = ok && c >= buf[1][col + 1] && c >= buf[2][col - 1] && c >= buf[2][col] && c >= buf[2][col + 1];
        flag[q] = ok;
        cnt += ok ? 1 : 0;
    }
    return cnt;
}

// Tiles per chunk (the unit of the per-chunk totals and offsets).
constexpr int kTilesPerBlock = 16;
// Workgroups of the count and write kernels (they stride over the chunks).
constexpr int kPeakGrid = 2048;

// Tile flags: flag[tile] = 1 iff the tile's row segment holds a cell above
// the threshold (only such tiles can hold a peak), and the chunk flag
// cflag[tile / 16] = 1 with it.  k_peak_mark streams the whole plane as one
// flat array in 16-byte vectors, four per thread in flight (any alignment of
// the plane pointer: a head and a tail of single cells), so the common empty
// tile costs one read of its cells and no neighbourhood.  k_peak_clear
// zeroes both flag arrays (n entries, stored back to back) at the start of
// every call (a kernel, not a memset, so the call can be captured in a
// graph).
__global__ void k_peak_clear(uint8_t *flags, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = 0;
}

template <class PT>
__device__ __forceinline__ void mark_cell(const PT *plane, int64_t f, int64_t n, int64_t n_cb, double thr,
                                          uint8_t *flags, uint8_t *cflags) {
    if (plane_val<PT>(plane, f) > thr) {
        const int64_t z = f / n, col = f - z * n;
        const int64_t tile = z * n_cb + col / kPeakTileCols;
        flags[tile] = 1;
        cflags[tile / kTilesPerBlock] = 1;
    }
}

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));

// Could the 16-byte vector u hold a cell above the threshold?  A superset
// test (exact test in mark_cell).  Raw bfloat16 with thr >= 0: a cell above
// thr has a bit pattern above tb, the pattern of thr truncated to bfloat16
// (patterns of non-negative values order like the values; negative values
// and NaN have larger patterns and are rechecked), four packed 16-bit
// maxima.  Other types, or thr < 0 / NaN: the exact comparison.
template <class PT>
__device__ __forceinline__ bool maybe_above(const u32x4_t &u, double thr, unsigned short tb, bool use_bits) {
    constexpr int kVec = 16 / sizeof(PT);
    if constexpr (sizeof(PT) == 2) {
        if (use_bits) {
            // words copied to scalars first: a bit cast of a vector element
            // expression (u.y) reads the vector's first element with this
            // compiler
            const uint32_t w0 = u.x, w1 = u.y, w2 = u.z, w3 = u.w;
            const u16x2_t m = __builtin_elementwise_max(
                __builtin_elementwise_max(__builtin_bit_cast(u16x2_t, w0), __builtin_bit_cast(u16x2_t, w1)),
                __builtin_elementwise_max(__builtin_bit_cast(u16x2_t, w2), __builtin_bit_cast(u16x2_t, w3)));
            return (m.x > tb) | (m.y > tb);
        }
    }
    const PT *cells = reinterpret_cast<const PT *>(&u);
    bool any = false;
#pragma unroll
    for (int q = 0; q < kVec; ++q) any |= plane_val<PT>(cells, q) > thr;
    return any;
}

template <class PT>
__global__ void __launch_bounds__(256) k_peak_mark(const PT *plane, int64_t n, int64_t total, int64_t n_cb, float thr_f,
                                                   uint8_t *flags, uint8_t *cflags) {
    constexpr int kVec = 16 / sizeof(PT);   // cells per 16-byte vector
    constexpr int kUnroll = 4;              // vectors in flight per thread
    const double thr = (double)thr_f;
    const bool use_bits = thr_f >= 0.0f;    // false for NaN too
    const unsigned short tb = (unsigned short)(__float_as_uint(thr_f) >> 16);
    const uintptr_t addr = reinterpret_cast<uintptr_t>(plane);
    int64_t head = (int64_t)(((16 - (addr & 15)) & 15) / sizeof(PT));
    if (head > total) head = total;
    const int64_t n_vec = (total - head) / kVec;
    const int64_t tail0 = head + n_vec * kVec;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (gid < head) mark_cell<PT>(plane, gid, n, n_cb, thr, flags, cflags);
    if (gid < total - tail0) mark_cell<PT>(plane, tail0 + gid, n, n_cb, thr, flags, cflags);
    const u32x4_t *vp = reinterpret_cast<const u32x4_t *>(plane + head);
    for (int64_t v0 = gid; v0 < n_vec; v0 += kUnroll * stride) {
        u32x4_t u[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int64_t v = v0 + k * stride;
            u[k] = v < n_vec ? __builtin_nontemporal_load(vp + v) : u32x4_t{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int64_t v = v0 + k * stride;
            if (v < n_vec && maybe_above<PT>(u[k], thr, tb, use_bits)) {   // rare: locate the cells
#pragma unroll
                for (int q = 0; q < kVec; ++q)
                    mark_cell<PT>(plane, head + v * kVec + q, n, n_cb, thr, flags, cflags);
            }
        }
    }
}

template <class PT>
__global__ void __launch_bounds__(kPeakThreads)
k_peak_count(const PT *plane, int64_t n, int n_z, int64_t n_cb, int64_t n_tiles, float thr, const uint8_t *flags,
             const uint8_t *cflags, int32_t *counts, int32_t *block_counts) {
    __shared__ peak_val_t<PT> buf[3][kPeakTileCols + 2];
    __shared__ int sum;
    const int64_t n_chunks = (n_tiles + kTilesPerBlock - 1) / kTilesPerBlock;
    for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
        if (cflags[ch] == 0) {                   // uniform: no cell above the threshold in the chunk
            if (threadIdx.x == 0) block_counts[ch] = 0;
            continue;
        }
        int total = 0;   // thread 0: peaks of this chunk's tiles
        for (int i = 0; i < kTilesPerBlock; ++i) {
            const int64_t tile = ch * kTilesPerBlock + i;
            if (tile >= n_tiles) break;
            if (flags[tile] == 0) continue;      // uniform; its count is never read
            const int z = (int)(tile / n_cb);
            const int64_t c0 = (tile % n_cb) * kPeakTileCols;
            if (threadIdx.x == 0) sum = 0;       // visible after the barrier inside tile_flags
            bool flag[kCellsPerThread];
            const int cnt = tile_flags<PT>(plane, n, n_z, z, c0, thr, buf, flag);
            if (cnt) atomicAdd(&sum, cnt);
            __syncthreads();
            if (threadIdx.x == 0) {
                counts[tile] = sum;
                total += sum;
            }
            __syncthreads();                     // buf and sum are reused by the next tile
        }
        if (threadIdx.x == 0) block_counts[ch] = total;
    }
}

// Single workgroup: exclusive scan of the per-workgroup totals -> offsets,
// total -> *n_found (kTilesPerBlock times fewer entries than tiles).
__global__ void __launch_bounds__(1024) k_peak_scan(const int32_t *counts, int64_t *offsets, int64_t n_tiles,
                                                    int64_t *n_found) {
    __shared__ int64_t part[1024];
    const int64_t per = (n_tiles + 1023) / 1024;
    const int64_t b = threadIdx.x * per;
    const int64_t e = min(b + per, n_tiles);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 partial sums
    for (int w = 1; w < 1024; w <<= 1) {
        const int64_t v = threadIdx.x >= (unsigned)w ? part[threadIdx.x - w] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int64_t i = b; i < e; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (threadIdx.x == 1023) *n_found = part[1023];
}

// Recompute the flags of one tile that holds peaks and write them at the
// tile's offset in column order, dropping those at or beyond the capacity.
template <class PT>
__device__ __forceinline__ void write_tile(const PT *plane, int64_t n, int n_z, int64_t n_cb, int64_t tile,
                                           float thr, int64_t tile_off, fdas_peak *out, int64_t capacity,
                                           peak_val_t<PT> (*buf)[kPeakTileCols + 2], int *pre) {
    const int z = (int)(tile / n_cb);
    const int64_t c0 = (tile % n_cb) * kPeakTileCols;
    bool flag[kCellsPerThread];
    const int cnt = tile_flags<PT>(plane, n, n_z, z, c0, thr, buf, flag);
    pre[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = 1; w < kPeakThreads; w <<= 1) {
        const int v = threadIdx.x >= (unsigned)w ? pre[threadIdx.x - w] : 0;
        __syncthreads();
        pre[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t pos = tile_off + pre[threadIdx.x] - cnt;
#pragma unroll
    for (int q = 0; q < kCellsPerThread; ++q) {
        if (!flag[q]) continue;
        if (pos < capacity) {
            const int col = threadIdx.x * kCellsPerThread + q + 1;
            fdas_peak pk;
            pk.r = c0 + col - 1;
            pk.z_idx = z;
            pk.job = 0;
            pk.power = (float)buf[1][col];
            pk.reserved = 0.0f;
            out[pos] = pk;
        }
        ++pos;
    }
}

template <class PT>
__global__ void __launch_bounds__(kPeakThreads)
k_peak_write(const PT *plane, int64_t n, int n_z, int64_t n_cb, int64_t n_tiles, float thr, const uint8_t *flags,
             const int32_t *counts, const int32_t *block_counts, const int64_t *block_offsets, fdas_peak *out,
             int64_t capacity) {
    __shared__ peak_val_t<PT> buf[3][kPeakTileCols + 2];
    __shared__ int pre[kPeakThreads];
    const int64_t n_chunks = (n_tiles + kTilesPerBlock - 1) / kTilesPerBlock;
    for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
        if (block_counts[ch] == 0) continue;     // uniform: no peak in the chunk
        int64_t off = block_offsets[ch];
        for (int i = 0; i < kTilesPerBlock; ++i) {
            const int64_t tile = ch * kTilesPerBlock + i;
            if (tile >= n_tiles) break;
            if (flags[tile] == 0) continue;      // uniform: counts[tile] was not written
            const int cnt = counts[tile];
            if (cnt == 0) continue;              // uniform: no peak in this tile
            write_tile<PT>(plane, n, n_z, n_cb, tile, thr, off, out, capacity, buf, pre);
            off += cnt;
            __syncthreads();                     // buf and pre are reused by the next tile
        }
    }
}

namespace {
template <class PT>
hipError_t run(const fdas_plan_s &p, const PT *plane, int64_t n, float thr, fdas_peak *out, int64_t cap,
               int64_t *n_found, hipStream_t st) {
    const int64_t n_cb = (n + kPeakTileCols - 1) / kPeakTileCols;
    const int64_t n_tiles = n_cb * p.cfg.n_z;
    if (n_tiles > p.peak_tile_cap || n_tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    unsigned char *scr = static_cast<unsigned char *>(p.ws) + p.off_scr;
    const int64_t n_blocks = (n_tiles + kTilesPerBlock - 1) / kTilesPerBlock;     // chunks
    int64_t *offsets = reinterpret_cast<int64_t *>(scr);                           // per chunk
    int32_t *counts = reinterpret_cast<int32_t *>(scr + (size_t)n_blocks * sizeof(int64_t));   // per tile
    int32_t *block_counts = counts + n_tiles;                                       // per chunk
    uint8_t *flags = reinterpret_cast<uint8_t *>(block_counts + n_blocks);            // per tile
    uint8_t *cflags = flags + n_tiles;                                              // per chunk
    const unsigned grid = (unsigned)std::min<int64_t>(n_blocks, kPeakGrid);
    const int64_t total = n_tiles / n_cb * n;                                       // cells of the plane
    hipLaunchKernelGGL(k_peak_clear, dim3((unsigned)std::min<int64_t>((n_tiles + n_blocks + 255) / 256, 4096)),
                       dim3(256), 0, st, flags, n_tiles + n_blocks);
    hipLaunchKernelGGL(k_peak_mark<PT>, dim3(8192), dim3(256), 0, st, plane, n, total, n_cb, thr, flags, cflags);
    hipLaunchKernelGGL(k_peak_count<PT>, dim3(grid), dim3(kPeakThreads), 0, st, plane, n, p.cfg.n_z, n_cb, n_tiles,
                       thr, flags, cflags, counts, block_counts);
    hipLaunchKernelGGL(k_peak_scan, dim3(1), dim3(1024), 0, st, block_counts, offsets, n_blocks, n_found);
    hipLaunchKernelGGL(k_peak_write<PT>, dim3(grid), dim3(kPeakThreads), 0, st, plane, n, p.cfg.n_z, n_cb, n_tiles,
                       thr, flags, counts, block_counts, offsets, out, cap);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_peaks(const fdas_plan_s &p, const void *plane, int64_t n, float thr, fdas_peak *out,
                        int64_t capacity, int64_t *n_found, hipStream_t st) {
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32: return run<float>(p, static_cast<const float *>(plane), n, thr, out, capacity, n_found, st);
        case FDAS_BF16:
            return run<unsigned short>(p, static_cast<const unsigned short *>(plane), n, thr, out, capacity,
                                       n_found, st);
        case FDAS_FP64: return run<double>(p, static_cast<const double *>(plane), n, thr, out, capacity, n_found, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdas
