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
//   count  a fixed grid of workgroups, each owning a contiguous range of
//          chunks: it reads 256 chunk flags at a time in one coalesced load,
//          lists the flagged ones in order (wave ballots), counts the peaks
//          of their flagged tiles and sums them into one total per workgroup;
//   scan   one workgroup turns the (at most 2048) workgroup totals into
//          exclusive offsets and the total;
//   write  the same ranges again: each workgroup walks its flagged chunks in
//          order from its offset, recomputes the peaks of tiles that have
//          any and writes them in column order, dropping those at or beyond
//          the capacity.
// A plane with few peaks thus costs one streaming read plus two passes over
// one byte per chunk, and no launch walks a long list serially.  The list is
// sorted by (z_idx, r) with no sort pass.
//
#include <algorithm>
#include <type_traits>

#include "internal.hpp"
#include "marks.hpp"

namespace fdas {

constexpr int kPeakThreads = 256;
constexpr int kCellsPerThread = kPeakTileCols / kPeakThreads;   // 4

// Workgroups of the count and write kernels (each takes every kPeakGrid-th
// range of chunks).
constexpr int kPeakGrid = kBatchPeakGrid;

// counts (int32) and flags (uint8) per tile, totals (int32) and flags per
// chunk of 16 tiles, totals and offsets per chunk range, with padding
size_t peak_scratch_bytes(int64_t n_tiles) {
    return (size_t)n_tiles * 6 + (size_t)kPeakRanges * (sizeof(int32_t) + sizeof(int64_t)) + 4096;
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

// Cells of a stored plane (n columns per row).  stage() fills buf with
// rows z-1..z+1, columns c0-1 .. c0+kPeakTileCols (-inf outside the n_c
// columns and n_z rows).
template <class PT>
struct PlaneCells {
    using V = peak_val_t<PT>;
    const PT *plane;
    int64_t n;
    __device__ __forceinline__ void stage(V (*buf)[kPeakTileCols + 2], int64_t n_c, int n_z, int z,
                                          int64_t c0) const {
        for (int i = threadIdx.x; i < 3 * (kPeakTileCols + 2); i += kPeakThreads) {
            const int row = i / (kPeakTileCols + 2);
            const int col = i % (kPeakTileCols + 2);
            const int zz = z + row - 1;
            const int64_t cc = c0 + col - 1;
            V v = -INFINITY;
            if (zz >= 0 && zz < n_z && cc >= 0 && cc < n_c) v = (V)plane_val<PT>(plane, (int64_t)zz * n + cc);
            buf[row][col] = v;
        }
    }
};

template <class Cells>
__device__ __forceinline__ int tile_flags(const Cells &cells, int64_t n, int n_z, int z, int64_t c0, float thr_f,
                                          typename Cells::V (*buf)[kPeakTileCols + 2], bool *flag) {
    using V = typename Cells::V;
    const V thr = (V)thr_f;
    cells.stage(buf, n, n_z, z, c0);
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

// Tiles per chunk (the unit of the per-chunk totals).
constexpr int kTilesPerBlock = kPeakTilesPerChunk;

// Tile flags: flag[tile] = 1 iff the tile's row segment holds a cell above
// the threshold (only such tiles can hold a peak), and the chunk flag
// cflag[tile / 16] = 1 with it.  k_peak_mark streams the whole plane as one
// flat array in 16-byte vectors, four per thread in flight (any alignment of
// the plane pointer: a head and a tail of single cells), so the common empty
// tile costs one read of its cells and no neighbourhood.  k_peak_clear
// zeroes both flag arrays (n entries, stored back to back) at the start of
// every call (a kernel, not a memset, so the call can be captured in a
// graph).  A marking correlation sets the same flags while it stores the
// plane (marks.hpp); the mark pass is then skipped.
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

// Could the 16-byte vector u hold a cell above the threshold?  A superset
// test (exact test in mark_cell): raw bfloat16 through the packed bit-pattern
// maximum of marks.hpp, other types the exact comparison.
template <class PT>
__device__ __forceinline__ bool maybe_above(const u32x4_t &u, double thr, const PeakMarks &m) {
    constexpr int kVec = 16 / sizeof(PT);
    if constexpr (sizeof(PT) == 2) {
        const uint32_t w0 = u.x, w1 = u.y, w2 = u.z, w3 = u.w;   // scalars first (see marks.hpp)
        return bf16x8_maybe_above(w0, w1, w2, w3, m);
    }
    const PT *cells = reinterpret_cast<const PT *>(&u);
    bool any = false;
#pragma unroll
    for (int q = 0; q < kVec; ++q) any |= plane_val<PT>(cells, q) > thr;
    return any;
}

// total cells of the plane; m.flags / m.cflags / m.n_cb / m.thr describe it
template <class PT>
__global__ void __launch_bounds__(256) k_peak_mark(const PT *plane, int64_t n, int64_t total, PeakMarks m) {
    constexpr int kVec = 16 / sizeof(PT);   // cells per 16-byte vector
    constexpr int kUnroll = 4;              // vectors in flight per thread
    const double thr = (double)m.thr;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(plane);
    int64_t head = (int64_t)(((16 - (addr & 15)) & 15) / sizeof(PT));
    if (head > total) head = total;
    const int64_t n_vec = (total - head) / kVec;
    const int64_t tail0 = head + n_vec * kVec;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (gid < head) mark_cell<PT>(plane, gid, n, m.n_cb, thr, m.flags, m.cflags);
    if (gid < total - tail0) mark_cell<PT>(plane, tail0 + gid, n, m.n_cb, thr, m.flags, m.cflags);
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
            if (v < n_vec && maybe_above<PT>(u[k], thr, m)) {   // rare: locate the cells
#pragma unroll
                for (int q = 0; q < kVec; ++q)
                    mark_cell<PT>(plane, head + v * kVec + q, n, m.n_cb, thr, m.flags, m.cflags);
            }
        }
    }
}

// Peaks of the flagged tiles of chunk ch of one plane (n_tiles tiles of
// n_cb per row): counts[tile] for each flagged tile; returns the chunk's
// total on thread 0.  Called by the whole workgroup; contains barriers.
template <class Cells>
__device__ __forceinline__ int count_chunk(const Cells &cells, int64_t n, int n_z, int64_t n_cb, int64_t n_tiles,
                                           int64_t ch, float thr, const uint8_t *flags, int32_t *counts,
                                           typename Cells::V (*buf)[kPeakTileCols + 2], int *sum) {
    int total = 0;   // thread 0: peaks of this chunk's tiles
    for (int i = 0; i < kTilesPerBlock; ++i) {
        const int64_t tile = ch * kTilesPerBlock + i;
        if (tile >= n_tiles) break;
        if (flags[tile] == 0) continue;      // uniform; its count is never read
        const int z = (int)(tile / n_cb);
        const int64_t c0 = (tile % n_cb) * kPeakTileCols;
        if (threadIdx.x == 0) *sum = 0;      // visible after the barrier inside tile_flags
        bool flag[kCellsPerThread];
        const int cnt = tile_flags(cells, n, n_z, z, c0, thr, buf, flag);
        if (cnt) atomicAdd(sum, cnt);
        __syncthreads();
        if (threadIdx.x == 0) {
            counts[tile] = *sum;
            total += *sum;
        }
        __syncthreads();                     // buf and sum are reused by the next tile
    }
    return total;
}

// Flagged chunks among [c0, c0 + kPeakThreads) (below c_end), listed in
// increasing order into list[] (offsets from c0); returns their number.
// One coalesced byte load per thread and a ballot per wave.  Called by the
// whole workgroup; contains barriers.
__device__ __forceinline__ int flagged_chunks(const uint8_t *cflags, int64_t c0, int64_t c_end, int *list,
                                              int *wave_cnt) {
    constexpr int kWaves = kPeakThreads / 64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool f = c0 + t < c_end && cflags[c0 + t] != 0;
    const uint64_t bal = __ballot(f);
    if (lane == 0) wave_cnt[w] = __popcll(bal);
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        base += i < w ? wave_cnt[i] : 0;
        total += wave_cnt[i];
    }
    if (f) list[base + __popcll(bal & ((1ull << lane) - 1ull))] = t;
    __syncthreads();
    return total;
}

// Chunk range v of n_ranges: [v per, min((v + 1) per, n_chunks)).
__device__ __forceinline__ void chunk_range(int64_t n_chunks, int64_t n_ranges, int64_t v, int64_t *r0,
                                            int64_t *r1) {
    const int64_t per = (n_chunks + n_ranges - 1) / n_ranges;
    *r0 = v * per;
    *r1 = min(*r0 + per, n_chunks);
}

// Job of chunk ch of a batch: the last job whose first chunk is <= ch.
__device__ __forceinline__ int job_of_chunk(const fdas_batch_job *jobs, int n_jobs, int64_t ch) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].chunk_base <= ch) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Where the chunks of a plane live: one plane, or a batch (chunk ch belongs
// to job job_of_chunk(ch), whose tiles start at its tile_base).
// A chunk's place: its cells, its plane's width and tiles, the chunk index
// inside that plane, the plane's first tile, the threshold, the list it
// writes to (slot) and the job its records name.
template <class Cells>
struct ChunkLocal {
    Cells cells;
    int64_t n, n_cb, n_tiles, ch, tile_base;
    float thr;
    int slot, job;
};

template <class PT>
struct ChunkSource {
    using Cells = PlaneCells<PT>;
    using V = peak_val_t<PT>;
    const PT *plane;                  // single plane / the batch's planes buffer
    int64_t n, n_cb, n_tiles;         // single plane
    const fdas_batch_job *jobs;       // batch (null for a single plane)
    int n_jobs;
    float thr;

    __device__ __forceinline__ ChunkLocal<Cells> at(int64_t ch, int n_z) const {
        if (!jobs) return ChunkLocal<Cells>{Cells{plane, n}, n, n_cb, n_tiles, ch, 0, thr, 0, 0};
        const int jb = job_of_chunk(jobs, n_jobs, ch);
        const int64_t nb = jobs[jb].n_bins;
        const int64_t cb = (nb + kPeakTileCols - 1) / kPeakTileCols;
        return ChunkLocal<Cells>{Cells{plane + jobs[jb].plane_off, nb}, nb, cb, cb * n_z, ch - jobs[jb].chunk_base,
                                 jobs[jb].tile_base, thr, jb, jb};
    }
};

// Cells of a harmonic sum that is never stored: S_H[z, r] = sum_{h <= H}
// P[z_h, h r] over the job's plane, added in the order h = 1, 2, ... in the
// summing kernel's precision and rounded to the plane's type as its store
// would be, so every cell is bitwise the value the sum would hold.  rows:
// [n_z][hmax] harmonic rows (-1: off the grid).  stage() takes the
// harmonics in the outer loop and the three template rows and the thread's
// cells inside it; no load sits behind a branch (a cell left out reads the
// row's first cell and keeps its sum), so the 15 loads of a harmonic are in
// flight together and a tile costs about H memory round trips.  A load is
// a buffer load (the row as a resource, a 32-bit byte offset) when a row
// holds less than 4 GB.
template <class PT>
struct SumCells {
    using V = peak_val_t<PT>;
    const PT *plane;
    int64_t n;                        // the job's bins (plane row length)
    const int32_t *rows;
    int hmax, H;

    __device__ __forceinline__ static V load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        if constexpr (sizeof(PT) == 8)
            return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
        else if constexpr (sizeof(PT) == 4)
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
        else
            return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0) << 16);
    }

    __device__ __forceinline__ void stage(V (*buf)[kPeakTileCols + 2], int64_t n_c, int n_z, int z,
                                          int64_t c0) const {
        constexpr int W = kPeakTileCols + 2;
        constexpr int Q = (W + kPeakThreads - 1) / kPeakThreads;        // cells per thread and row
        const bool wide = n >= (int64_t)(0xffffffffu / sizeof(PT));
        const int32_t row_bytes = (int32_t)(uint32_t)(n * (int64_t)sizeof(PT));
        V acc[3][Q];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[k][q] = V(0);
        for (int h = 1; h <= H; ++h) {
            int jr[3];
            V v[3][Q];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int zz = z + k - 1;
                jr[k] = (zz >= 0 && zz < n_z) ? __builtin_amdgcn_readfirstlane(rows[zz * hmax + h - 1]) : -1;
                const PT *base = plane + (int64_t)max(jr[k], 0) * n;
                const __amdgpu_buffer_rsrc_t rs =
                    __builtin_amdgcn_make_buffer_rsrc(const_cast<PT *>(base), (short)0, row_bytes, 0x00020000);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int x = threadIdx.x + q * kPeakThreads;
                    const int64_t col = c0 - 1 + x;
                    const bool ok = x < W && jr[k] >= 0 && col >= 0 && col < n_c;
                    if (!wide) {
                        v[k][q] = load(rs, ok ? (uint32_t)h * (uint32_t)col * (uint32_t)sizeof(PT) : 0u);
                    } else {
                        v[k][q] = (V)plane_val<PT>(base, ok ? (int64_t)h * col : 0);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int x = threadIdx.x + q * kPeakThreads;
                    const int64_t col = c0 - 1 + x;
                    const bool ok = x < W && jr[k] >= 0 && col >= 0 && col < n_c;
                    acc[k][q] = ok ? acc[k][q] + v[k][q] : acc[k][q];
                }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int x = threadIdx.x + q * kPeakThreads;
                if (x >= W) continue;
                const int zz = z + k - 1;
                const int64_t col = c0 - 1 + x;
                V val = -INFINITY;
                if (zz >= 0 && zz < n_z && col >= 0 && col < n_c) {
                    if constexpr (sizeof(PT) == 2) val = (float)(__bf16)acc[k][q];   // the bfloat16 store, widened
                    else val = acc[k][q];
                }
                buf[k][x] = val;
            }
    }
};

template <class PT>
struct SumSource {
    using Cells = SumCells<PT>;
    using V = peak_val_t<PT>;
    const PT *planes;
    const fdas_batch_job *jobs;
    const SumJob *lists;
    int n_lists;
    const int32_t *rows;
    int hmax;

    __device__ __forceinline__ ChunkLocal<Cells> at(int64_t ch, int n_z) const {
        int lo = 0, hi = n_lists - 1;   // the last list whose first chunk is <= ch
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lists[mid].chunk_base <= ch) lo = mid;
            else hi = mid - 1;
        }
        const SumJob &sj = lists[lo];
        const fdas_batch_job &jb = jobs[sj.job];
        const int64_t cb = (sj.nh + kPeakTileCols - 1) / kPeakTileCols;
        return ChunkLocal<Cells>{Cells{planes + jb.plane_off, jb.n_bins, rows, hmax, sj.H}, sj.nh, cb, cb * n_z,
                                 ch - sj.chunk_base, sj.tile_base, sj.thr, lo, sj.job};
    }
};

// Count: per flagged chunk its total (block_counts), per chunk range the sum
// (range_totals), per job the sum (job_totals, batch only: one atomic per
// chunk with peaks, zeroed with the flags).
template <class Src>
__global__ void __launch_bounds__(kPeakThreads)
k_peak_count(Src src, int n_z, int64_t n_chunks, int64_t n_ranges, const uint8_t *flags, const uint8_t *cflags,
             int32_t *counts, int32_t *block_counts, int32_t *range_totals, unsigned long long *job_totals) {
    __shared__ typename Src::V buf[3][kPeakTileCols + 2];
    __shared__ int sum, list[kPeakThreads], wave_cnt[kPeakThreads / 64];
    for (int64_t v = blockIdx.x; v < n_ranges; v += gridDim.x) {
        int64_t r0, r1;
        chunk_range(n_chunks, n_ranges, v, &r0, &r1);
        int total = 0;   // thread 0
        for (int64_t c0 = r0; c0 < r1; c0 += kPeakThreads) {
            const int nf = flagged_chunks(cflags, c0, r1, list, wave_cnt);
            for (int k = 0; k < nf; ++k) {
                const int64_t ch = c0 + list[k];
                const auto loc = src.at(ch, n_z);
                const int t = count_chunk(loc.cells, loc.n, n_z, loc.n_cb, loc.n_tiles, loc.ch, loc.thr,
                                          flags + loc.tile_base, counts + loc.tile_base, buf, &sum);
                if (threadIdx.x == 0) {
                    block_counts[ch] = t;
                    total += t;
                    if (job_totals && t) atomicAdd(&job_totals[loc.slot], (unsigned long long)t);
                }
            }
            __syncthreads();                     // list is rewritten by the next group
        }
        if (threadIdx.x == 0) range_totals[v] = total;
    }
}

// Exclusive scan of n values by one workgroup of 1024 threads: offsets[i] =
// vals[0] + .. + vals[i - 1] (int64), copy[i] = vals[i] when copy is not
// null; returns the total.  Thread t takes the run [t per, t per + per), per
// = ceil(n / 1024) rounded up to a multiple of 4.  For 32-bit values and
// runs of up to kScanRegs inside the array, the run is read as 16-byte loads
// from one address, all in flight together, and written back from the
// registers, so it costs one memory round trip instead of one per value;
// other runs are summed and written by loops.  part: 32 int64 of LDS.
constexpr int kScanRegs = 32;

template <class T>
__device__ int64_t block_exclusive_scan(const T *vals, int64_t n, int64_t *offsets, int64_t *copy, int64_t *part) {
    const int64_t per = (((n + 1023) / 1024) + 3) & ~(int64_t)3;
    const int64_t b = threadIdx.x * per;
    const int64_t e = min(b + per, n);
    constexpr bool kWide = sizeof(T) == 4;
    const bool wide = kWide && per <= kScanRegs && b + per <= n &&
                      (reinterpret_cast<uintptr_t>(vals) % 16) == 0;   // whole run, 16-byte aligned
    uint32_t v[kScanRegs];
    int64_t s = 0;
    __syncthreads();   // part may still be read from a previous scan
    if (wide) {
        const uint4 *q = reinterpret_cast<const uint4 *>(vals + b);
#pragma unroll
        for (int i = 0; i < kScanRegs / 4; ++i) {
            if (4 * i < per) {
                const uint4 u = q[i];
                v[4 * i] = u.x;
                v[4 * i + 1] = u.y;
                v[4 * i + 2] = u.z;
                v[4 * i + 3] = u.w;
            }
        }
#pragma unroll
        for (int i = 0; i < kScanRegs; ++i)
            if (i < per) s += (int64_t)(T)v[i];
    } else {
        for (int64_t i = b; i < e; ++i) s += (int64_t)vals[i];
    }
    // inclusive scan of the 1024 partial sums: within each wave by shuffles,
    // then over the 16 wave totals (part[0 .. 15]) by the first wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t x = __shfl_up(incl, o, 64);
        if (lane >= o) incl += x;
    }
    if (lane == 63) part[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        int64_t t = lane < 16 ? part[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int64_t x = __shfl_up(t, o, 64);
            if (lane >= o) t += x;
        }
        if (lane < 16) part[16 + lane] = t;   // inclusive prefix of the wave totals
    }
    __syncthreads();
    int64_t run = (wave ? part[16 + wave - 1] : 0) + incl - s;   // exclusive prefix of this thread's run
    const int64_t total = part[16 + 15];
    if (wide) {
        int64_t *o = offsets + b;
#pragma unroll
        for (int i = 0; i < kScanRegs; ++i) {
            if (i < per) {
                const int64_t x = (int64_t)(T)v[i];
                o[i] = run;
                if (copy) copy[b + i] = x;
                run += x;
            }
        }
    } else {
        for (int64_t i = b; i < e; ++i) {
            const int64_t x = (int64_t)vals[i];
            offsets[i] = run;
            if (copy) copy[i] = x;
            run += x;
        }
    }
    return total;
}

// Single workgroup: exclusive scan of n >= 1 values -> offsets[0 .. n)
// (int64), the total -> offsets[n] and *total; with copy != null the values
// are also copied there (per-job counts of a batch).
template <class T>
__global__ void __launch_bounds__(1024) k_peak_scan(const T *vals, int64_t n, int64_t *offsets, int64_t *total,
                                                    int64_t *copy) {
    __shared__ int64_t part[32];
    const int64_t t = block_exclusive_scan(vals, n, offsets, copy, part);
    if (threadIdx.x == 1023) {
        offsets[n] = t;
        *total = t;
    }
}

// Recompute the flags of one tile that holds peaks and write them at the
// tile's offset in column order, dropping those at or beyond the capacity.
template <class Cells>
__device__ __forceinline__ void write_tile(const Cells &cells, int64_t n, int n_z, int64_t n_cb, int64_t tile,
                                           float thr, int64_t tile_off, fdas_peak *out, int64_t capacity, int job,
                                           typename Cells::V (*buf)[kPeakTileCols + 2], int *pre) {
    const int z = (int)(tile / n_cb);
    const int64_t c0 = (tile % n_cb) * kPeakTileCols;
    bool flag[kCellsPerThread];
    const int cnt = tile_flags(cells, n, n_z, z, c0, thr, buf, flag);
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
            pk.job = job;
            pk.power = (float)buf[1][col];
            pk.reserved = 0.0f;
            out[pos] = pk;
        }
        ++pos;
    }
}

// The peaks of chunk ch of one plane, written from offset off on.  Called by
// the whole workgroup; contains barriers.
template <class Cells>
__device__ __forceinline__ void write_chunk(const Cells &cells, int64_t n, int n_z, int64_t n_cb, int64_t n_tiles,
                                            int64_t ch, float thr, const uint8_t *flags, const int32_t *counts,
                                            int64_t off, fdas_peak *out, int64_t capacity, int job,
                                            typename Cells::V (*buf)[kPeakTileCols + 2], int *pre) {
    for (int i = 0; i < kTilesPerBlock; ++i) {
        const int64_t tile = ch * kTilesPerBlock + i;
        if (tile >= n_tiles) break;
        if (flags[tile] == 0) continue;      // uniform: counts[tile] was not written
        const int cnt = counts[tile];
        if (cnt == 0) continue;              // uniform: no peak in this tile
        write_tile(cells, n, n_z, n_cb, tile, thr, off, out, capacity, job, buf, pre);
        off += cnt;
        __syncthreads();                     // buf and pre are reused by the next tile
    }
}

// Write: each workgroup walks the flagged chunks of each of its ranges in
// order from the range's offset; a batch job's list starts at out + job *
// capacity and its offsets at the job's prefix (job_prefix).
template <class Src>
__global__ void __launch_bounds__(kPeakThreads)
k_peak_write(Src src, int n_z, int64_t n_chunks, int64_t n_ranges, const uint8_t *flags, const uint8_t *cflags,
             const int32_t *counts, const int32_t *block_counts, const int64_t *range_offsets,
             const int64_t *job_prefix, fdas_peak *out, int64_t capacity) {
    __shared__ typename Src::V buf[3][kPeakTileCols + 2];
    __shared__ int pre[kPeakThreads], list[kPeakThreads], wave_cnt[kPeakThreads / 64];
    for (int64_t v = blockIdx.x; v < n_ranges; v += gridDim.x) {
        int64_t r0, r1;
        chunk_range(n_chunks, n_ranges, v, &r0, &r1);
        int64_t run = range_offsets[v];       // peaks of all chunks before this range
        if (range_offsets[v + 1] == run) continue;   // uniform: no peak in this range
        for (int64_t c0 = r0; c0 < r1; c0 += kPeakThreads) {
            const int nf = flagged_chunks(cflags, c0, r1, list, wave_cnt);
            for (int k = 0; k < nf; ++k) {
                const int64_t ch = c0 + list[k];
                const int cnt = block_counts[ch];
                if (cnt == 0) continue;          // uniform
                const auto loc = src.at(ch, n_z);
                const int64_t off = job_prefix ? run - job_prefix[loc.slot] : run;
                write_chunk(loc.cells, loc.n, n_z, loc.n_cb, loc.n_tiles, loc.ch, loc.thr, flags + loc.tile_base,
                            counts + loc.tile_base, off, out + (int64_t)loc.slot * capacity, capacity, loc.job, buf,
                            pre);
                run += cnt;
            }
            __syncthreads();                     // list is rewritten by the next group
        }
    }
}

namespace {

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

// Scratch of the single-plane finder in the plan's workspace.
struct PeakScratch {
    int64_t n_cb, n_tiles, n_chunks;
    int32_t *counts;         // per tile
    int32_t *block_counts;   // per chunk
    int32_t *wg_totals;      // per chunk range
    int64_t *wg_offsets;     // per chunk range, then the total
    uint8_t *flags;          // per tile
    uint8_t *cflags;         // per chunk (right after flags: one clear covers both)
};

bool plane_scratch(const fdas_plan_s &p, int64_t n, PeakScratch *o) {
    o->n_cb = (n + kPeakTileCols - 1) / kPeakTileCols;
    o->n_tiles = o->n_cb * p.cfg.n_z;
    if (o->n_tiles > p.peak_tile_cap || o->n_tiles > 0x7fffffffLL) return false;
    o->n_chunks = (o->n_tiles + kTilesPerBlock - 1) / kTilesPerBlock;
    unsigned char *b = static_cast<unsigned char *>(p.ws) + p.off_scr;
    size_t off = 0;
    o->wg_offsets = reinterpret_cast<int64_t *>(b + off);
    off = up256(off + (kPeakRanges + 1) * sizeof(int64_t));
    o->wg_totals = reinterpret_cast<int32_t *>(b + off);
    off = up256(off + kPeakRanges * sizeof(int32_t));
    o->counts = reinterpret_cast<int32_t *>(b + off);
    off = up256(off + (size_t)o->n_tiles * sizeof(int32_t));
    o->block_counts = reinterpret_cast<int32_t *>(b + off);
    off = up256(off + (size_t)o->n_chunks * sizeof(int32_t));
    o->flags = b + off;
    o->cflags = o->flags + o->n_tiles;
    return true;
}

void launch_clear(uint8_t *flags, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_peak_clear, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))),
                       dim3(256), 0, st, flags, n);
}

// Workgroups of a mark pass over `total` cells (16-byte vectors, four per thread).
unsigned mark_grid(int64_t total, size_t elem) {
    const int64_t vecs = total / (int64_t)(16 / elem);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (vecs + 1023) / 1024));
}

// Count, scan and write over n_chunks chunks (flags already set).
// Both scans of a batch in one workgroup: workgroup offsets, then the
// per-list prefixes and counts.
__global__ void __launch_bounds__(1024) k_peak_scan_batch(const int32_t *wg_totals, int64_t n_wg, int64_t *wg_offsets,
                                                          const unsigned long long *job_totals, int64_t n_lists,
                                                          int64_t *job_prefix, int64_t *n_found) {
    __shared__ int64_t part[32];
    const int64_t t = block_exclusive_scan(wg_totals, n_wg, wg_offsets, (int64_t *)nullptr, part);
    if (threadIdx.x == 1023) wg_offsets[n_wg] = t;
    block_exclusive_scan(job_totals, n_lists, job_prefix, n_found, part);
}

template <class Src>
void launch_finish(const Src &src, int n_z, int64_t n_chunks, const uint8_t *flags, const uint8_t *cflags,
                   int32_t *counts, int32_t *block_counts, int32_t *wg_totals, int64_t *wg_offsets,
                   unsigned long long *job_totals, int64_t n_lists, int64_t *job_prefix, int64_t *n_found,
                   fdas_peak *out, int64_t cap, hipStream_t st) {
    const int64_t n_ranges = std::max<int64_t>(1, std::min<int64_t>(n_chunks, kPeakRanges));
    const unsigned grid = (unsigned)std::min<int64_t>(n_ranges, kPeakGrid);
    hipLaunchKernelGGL(k_peak_count<Src>, dim3(grid), dim3(kPeakThreads), 0, st, src, n_z, n_chunks, n_ranges, flags,
                       cflags, counts, block_counts, wg_totals, job_totals);
    if (job_totals)   // range offsets, per-list prefixes and counts
        hipLaunchKernelGGL(k_peak_scan_batch, dim3(1), dim3(1024), 0, st, wg_totals, n_ranges, wg_offsets,
                           job_totals, n_lists, job_prefix, n_found);
    else              // range offsets; a single plane's total is its count
        hipLaunchKernelGGL(k_peak_scan<int32_t>, dim3(1), dim3(1024), 0, st, wg_totals, n_ranges, wg_offsets,
                           n_found, (int64_t *)nullptr);
    hipLaunchKernelGGL(k_peak_write<Src>, dim3(grid), dim3(kPeakThreads), 0, st, src, n_z, n_chunks, n_ranges, flags,
                       cflags, counts, block_counts, wg_offsets, job_prefix, out, cap);
}

template <class PT>
hipError_t run(const fdas_plan_s &p, const PT *plane, int64_t n, float thr, fdas_peak *out, int64_t cap,
               int64_t *n_found, bool premarked, hipStream_t st) {
    PeakScratch sc;
    if (!plane_scratch(p, n, &sc)) return hipErrorInvalidValue;
    if (!premarked) {
        const int64_t total = (int64_t)p.cfg.n_z * n;   // cells of the plane
        launch_clear(sc.flags, sc.n_tiles + sc.n_chunks, st);
        hipLaunchKernelGGL(k_peak_mark<PT>, dim3(mark_grid(total, sizeof(PT))), dim3(256), 0, st, plane, n, total,
                           make_peak_marks(sc.flags, sc.cflags, sc.n_cb, thr));
    }
    ChunkSource<PT> src{plane, n, sc.n_cb, sc.n_tiles, nullptr, 0, thr};
    launch_finish(src, p.cfg.n_z, sc.n_chunks, sc.flags, sc.cflags, sc.counts, sc.block_counts, sc.wg_totals,
                  sc.wg_offsets, nullptr, 0, nullptr, n_found, out, cap, st);
    return hipGetLastError();
}

// Scratch of the batched finder (caller memory, 256-byte aligned regions).
struct BatchScratch {
    int32_t *counts;                 // per tile of all jobs
    int32_t *block_counts;           // per chunk
    int32_t *wg_totals;              // per chunk range
    int64_t *wg_offsets;             // per chunk range, then the grand total
    int64_t *job_prefix;             // per job
    unsigned long long *job_totals;  // per job (zeroed with the flags, right before them)
    uint8_t *flags;                  // per tile
    uint8_t *cflags;                 // per chunk (right after flags)
    size_t bytes;
};

BatchScratch batch_scratch(const fdas_plan_s &p, void *base) {
    const size_t T = (size_t)p.batch_peak_tiles, C = (size_t)p.batch_peak_chunks, J = (size_t)p.batch_jobs;
    unsigned char *b = static_cast<unsigned char *>(base);
    BatchScratch o;
    size_t off = 0;
    o.counts = reinterpret_cast<int32_t *>(b + off);
    off = up256(off + T * sizeof(int32_t));
    o.block_counts = reinterpret_cast<int32_t *>(b + off);
    off = up256(off + C * sizeof(int32_t));
    o.wg_totals = reinterpret_cast<int32_t *>(b + off);
    off = up256(off + kPeakRanges * sizeof(int32_t));
    o.wg_offsets = reinterpret_cast<int64_t *>(b + off);
    off = up256(off + (kPeakRanges + 1) * sizeof(int64_t));
    o.job_prefix = reinterpret_cast<int64_t *>(b + off);
    off = up256(off + J * sizeof(int64_t));
    o.job_totals = reinterpret_cast<unsigned long long *>(b + off);
    o.flags = b + off + J * sizeof(unsigned long long);
    o.cflags = o.flags + T;
    off = up256(off + J * sizeof(unsigned long long) + T + C);
    o.bytes = off;
    return o;
}

template <class PT>
hipError_t run_batch_mark(const fdas_plan_s &p, const PT *planes, const PeakMarks &m, hipStream_t st) {
    for (const fdas_batch_job &j : p.batch_host) {
        const int64_t total = (int64_t)p.cfg.n_z * j.n_bins;
        hipLaunchKernelGGL(k_peak_mark<PT>, dim3(mark_grid(total, sizeof(PT))), dim3(256), 0, st,
                           planes + j.plane_off, j.n_bins, total,
                           make_peak_marks(m.flags + j.tile_base, m.cflags + j.chunk_base,
                                           (j.n_bins + kPeakTileCols - 1) / kPeakTileCols, m.thr));
    }
    return hipGetLastError();
}

template <class PT>
hipError_t run_batch_finish(const fdas_plan_s &p, const PT *planes, void *scratch, float thr, fdas_peak *out,
                            int64_t cap, int64_t *n_found, hipStream_t st) {
    const BatchScratch sc = batch_scratch(p, scratch);
    const auto *jobs = reinterpret_cast<const fdas_batch_job *>(static_cast<const unsigned char *>(p.ws) +
                                                               p.off_batch + p.batch_hdr);
    ChunkSource<PT> src{planes, 0, 0, 0, jobs, p.batch_jobs, thr};
    launch_finish(src, p.cfg.n_z, p.batch_peak_chunks, sc.flags, sc.cflags, sc.counts, sc.block_counts,
                  sc.wg_totals, sc.wg_offsets, sc.job_totals, p.batch_jobs, sc.job_prefix, n_found, out, cap, st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_peaks(const fdas_plan_s &p, const void *plane, int64_t n, float thr, fdas_peak *out,
                        int64_t capacity, int64_t *n_found, hipStream_t st, bool premarked) {
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32:
            return run<float>(p, static_cast<const float *>(plane), n, thr, out, capacity, n_found, premarked, st);
        case FDAS_BF16:
            return run<unsigned short>(p, static_cast<const unsigned short *>(plane), n, thr, out, capacity,
                                       n_found, premarked, st);
        case FDAS_FP64:
            return run<double>(p, static_cast<const double *>(plane), n, thr, out, capacity, n_found, premarked, st);
        default: return hipErrorInvalidValue;
    }
}

// Count, scan and write of one plane whose flags were set by a marking
// kernel, with the counters in caller memory (work: peak_work_bytes).
size_t peak_work_bytes(int64_t n_tiles) {
    const int64_t n_chunks = (n_tiles + kTilesPerBlock - 1) / kTilesPerBlock;
    return up256((kPeakRanges + 1) * sizeof(int64_t)) + up256(kPeakRanges * sizeof(int32_t)) +
           up256((size_t)n_tiles * sizeof(int32_t)) + up256((size_t)n_chunks * sizeof(int32_t));
}

template <class PT>
hipError_t finish_plane(const fdas_plan_s &p, const PT *plane, int64_t n, float thr, const uint8_t *flags,
                        const uint8_t *cflags, void *work, fdas_peak *out, int64_t cap, int64_t *n_found,
                        hipStream_t st) {
    const int64_t n_cb = (n + kPeakTileCols - 1) / kPeakTileCols;
    const int64_t n_tiles = n_cb * p.cfg.n_z;
    const int64_t n_chunks = (n_tiles + kTilesPerBlock - 1) / kTilesPerBlock;
    unsigned char *b = static_cast<unsigned char *>(work);
    size_t off = 0;
    auto *wg_offsets = reinterpret_cast<int64_t *>(b + off);
    off += up256((kPeakRanges + 1) * sizeof(int64_t));
    auto *wg_totals = reinterpret_cast<int32_t *>(b + off);
    off += up256(kPeakRanges * sizeof(int32_t));
    auto *counts = reinterpret_cast<int32_t *>(b + off);
    off += up256((size_t)n_tiles * sizeof(int32_t));
    auto *block_counts = reinterpret_cast<int32_t *>(b + off);
    ChunkSource<PT> src{plane, n, n_cb, n_tiles, nullptr, 0, thr};
    launch_finish(src, p.cfg.n_z, n_chunks, flags, cflags, counts, block_counts, wg_totals, wg_offsets, nullptr, 0,
                  nullptr, n_found, out, cap, st);
    return hipGetLastError();
}

hipError_t peaks_finish_plane(const fdas_plan_s &p, const void *plane, int64_t n, float thr, const uint8_t *flags,
                              const uint8_t *cflags, void *work, fdas_peak *out, int64_t capacity, int64_t *n_found,
                              hipStream_t st) {
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32:
            return finish_plane<float>(p, static_cast<const float *>(plane), n, thr, flags, cflags, work, out,
                                       capacity, n_found, st);
        case FDAS_BF16:
            return finish_plane<unsigned short>(p, static_cast<const unsigned short *>(plane), n, thr, flags, cflags,
                                                work, out, capacity, n_found, st);
        case FDAS_FP64:
            return finish_plane<double>(p, static_cast<const double *>(plane), n, thr, flags, cflags, work, out,
                                        capacity, n_found, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t peak_flags_clear(uint8_t *flags, int64_t n, hipStream_t st) {
    launch_clear(flags, n, st);
    return hipGetLastError();
}

hipError_t peak_marks(const fdas_plan_s &p, int64_t n, float thr, PeakMarks *marks, hipStream_t st) {
    PeakScratch sc;
    if (!plane_scratch(p, n, &sc)) return hipErrorInvalidValue;
    launch_clear(sc.flags, sc.n_tiles + sc.n_chunks, st);
    *marks = make_peak_marks(sc.flags, sc.cflags, sc.n_cb, thr);
    return hipGetLastError();
}

size_t batch_peak_scratch_bytes(const fdas_plan_s &p) { return batch_scratch(p, nullptr).bytes; }

hipError_t batch_peak_marks(const fdas_plan_s &p, void *scratch, float thr, PeakMarks *marks, hipStream_t st) {
    const BatchScratch sc = batch_scratch(p, scratch);
    // per-job totals, tile flags and chunk flags, stored back to back
    launch_clear(reinterpret_cast<uint8_t *>(sc.job_totals),
                 (int64_t)(p.batch_jobs * sizeof(unsigned long long)) + p.batch_peak_tiles + p.batch_peak_chunks, st);
    // n_cb differs per job: the marking kernels derive it from the job's length
    *marks = make_peak_marks(sc.flags, sc.cflags, 0, thr);
    return hipGetLastError();
}

hipError_t batch_peak_mark_pass(const fdas_plan_s &p, const void *planes, const PeakMarks &marks, hipStream_t st) {
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32: return run_batch_mark<float>(p, static_cast<const float *>(planes), marks, st);
        case FDAS_BF16:
            return run_batch_mark<unsigned short>(p, static_cast<const unsigned short *>(planes), marks, st);
        case FDAS_FP64: return run_batch_mark<double>(p, static_cast<const double *>(planes), marks, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_peaks_finish(const fdas_plan_s &p, const void *planes, void *scratch, float thr, fdas_peak *out,
                              int64_t capacity, int64_t *n_found, hipStream_t st) {
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32:
            return run_batch_finish<float>(p, static_cast<const float *>(planes), scratch, thr, out, capacity,
                                           n_found, st);
        case FDAS_BF16:
            return run_batch_finish<unsigned short>(p, static_cast<const unsigned short *>(planes), scratch, thr,
                                                    out, capacity, n_found, st);
        case FDAS_FP64:
            return run_batch_finish<double>(p, static_cast<const double *>(planes), scratch, thr, out, capacity,
                                            n_found, st);
        default: return hipErrorInvalidValue;
    }
}

template <class PT>
hipError_t run_batch_sums_finish(const fdas_plan_s &p, const SumBatch &sb, const BatchSumsLayout &L, const PT *planes,
                                 unsigned char *b, fdas_peak *out, int64_t cap, int64_t *n_found, hipStream_t st) {
    const fdas_batch_job *jobs = sb.dev;
    auto *totals = reinterpret_cast<unsigned long long *>(b + L.off_totals);
    uint8_t *flags = b + L.off_totals + (size_t)L.lists * 8;
    SumSource<PT> src{planes, jobs, reinterpret_cast<const SumJob *>(b + L.off_lists), (int)L.lists,
                      reinterpret_cast<const int32_t *>(b + L.off_rows), L.hmax};
    launch_finish(src, p.cfg.n_z, L.chunks, flags, flags + L.tiles, reinterpret_cast<int32_t *>(b + L.off_counts),
                  reinterpret_cast<int32_t *>(b + L.off_block_counts), reinterpret_cast<int32_t *>(b + L.off_wg_totals),
                  reinterpret_cast<int64_t *>(b + L.off_wg_offsets), totals, L.lists,
                  reinterpret_cast<int64_t *>(b + L.off_prefix), n_found, out, cap, st);
    return hipGetLastError();
}

hipError_t batch_sums_finish(const fdas_plan_s &p, const SumBatch &sb, const BatchSumsLayout &L, const void *planes,
                             void *scratch, fdas_peak *out, int64_t capacity, int64_t *n_found, hipStream_t st) {
    auto *b = static_cast<unsigned char *>(scratch);
    switch (p.cfg.plane_dtype) {
        case FDAS_FP32:
            return run_batch_sums_finish<float>(p, sb, L, static_cast<const float *>(planes), b, out, capacity,
                                                n_found, st);
        case FDAS_BF16:
            return run_batch_sums_finish<unsigned short>(p, sb, L, static_cast<const unsigned short *>(planes), b,
                                                         out, capacity, n_found, st);
        case FDAS_FP64:
            return run_batch_sums_finish<double>(p, sb, L, static_cast<const double *>(planes), b, out, capacity,
                                                 n_found, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdas
