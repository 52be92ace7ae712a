// Tile flags of the thresholded peak finder.  The finder only examines tiles
// (one plane row x kPeakTileCols columns) that are flagged, grouped in chunks
// of kPeakTilesPerChunk tiles, and tests every cell of those exactly; every
// tile that holds a cell above the threshold must be flagged, and flagging
// more only costs time.  The flags are set either by the finder's own
// streaming pass over the plane (exactly those tiles) or by a correlation
// kernel while it stores the plane (fused form: the plane is then not read
// back; runs of cells that pass a superset test are flagged whole).
#pragma once

#include "internal.hpp"

namespace fdas {

// Flags of one plane and the test that sets them.  Both flag arrays are
// zeroed before the plane is marked; a set byte is only ever written as 1, so
// concurrent writers need no atomics.
struct PeakMarks {
    uint8_t *flags;      // one byte per tile, tile = z * n_cb + column / kPeakTileCols
    uint8_t *cflags;     // one byte per chunk of kPeakTilesPerChunk consecutive tiles
    int32_t n_cb;        // tiles per row (tile counts of a plane stay below 2^31)
    int32_t tb;          // thr >= 0: bit pattern of thr truncated to bfloat16; else -1
    float thr;           // a cell is above the threshold iff its value (widened exactly) > thr
};

__host__ inline PeakMarks make_peak_marks(uint8_t *flags, uint8_t *cflags, int64_t n_cb, float thr) {
    PeakMarks m;
    m.flags = flags;
    m.cflags = cflags;
    m.n_cb = (int32_t)n_cb;
    m.thr = thr;
    uint32_t bits;
    static_assert(sizeof(bits) == sizeof(thr), "float is 32-bit");
    __builtin_memcpy(&bits, &thr, sizeof(bits));
    // thr < 0 or NaN: -1, so that the prefilter passes every run
    m.tb = thr >= 0.0f ? (int32_t)(bits >> 16) : -1;
    return m;
}

__device__ __forceinline__ void mark_tile(const PeakMarks &m, int64_t z, int64_t col) {
    const int64_t tile = z * m.n_cb + col / kPeakTileCols;
    m.flags[tile] = 1;
    m.cflags[tile / kPeakTilesPerChunk] = 1;
}

// Conservative form for a correlation kernel: flags the tiles of columns
// seg0 + a and seg0 + b (a <= b, both inside the plane row whose first tile
// is row_tile0, at most one tile apart).  Flagging a tile that holds no cell
// above the threshold only costs the finder a look at it, so a run of cells
// that may hold one is flagged whole.  32-bit indices (row and tile counts
// of a marked plane stay below 2^31), so each address is a scalar base plus
// one 32-bit lane offset.
__device__ __forceinline__ void mark_run(const PeakMarks &m, uint32_t row_tile0, int32_t seg0, int a, int b) {
    static_assert(kPeakTileCols == 1024, "tile index by shift");
    if (a > b) return;
    const uint32_t ta = row_tile0 + ((uint32_t)(seg0 + a) >> 10);
    const uint32_t tb = row_tile0 + ((uint32_t)(seg0 + b) >> 10);
    m.flags[ta] = 1;
    m.cflags[ta / kPeakTilesPerChunk] = 1;
    if (tb != ta) {
        m.flags[tb] = 1;
        m.cflags[tb / kPeakTilesPerChunk] = 1;
    }
}

// The harmonic-sum lists of a batch (fdas_batch_harmonic_sums_peaks): list
// l * n_jobs + i holds the peaks of job i's sum over H_l harmonics, a virtual
// plane of n_z x nh cells that is never stored (its flagged tiles are
// recomputed from the job's plane).  Tiles and chunks of all lists share one
// index space, lists in order.
struct SumJob {
    int64_t nh;          // columns of the sum (fundamentals r < N_H)
    int64_t tile_base;   // first tile among all lists' tiles
    int64_t chunk_base;  // first chunk
    int64_t block_base;  // lists of the first level: first workgroup of the summing kernel
    int32_t H, job;
    float thr;
    int32_t level;
};

// Largest row length a marking correlation accepts (32-bit columns with a
// segment of headroom).
constexpr int64_t kMarkMaxBins = ((int64_t)1 << 31) - 65536;

typedef unsigned short marks_u16x2_t __attribute__((ext_vector_type(2)));

// Could eight raw bfloat16 values (four packed words) hold one above thr?
// For thr >= 0 a value above thr has a bit pattern above tb (patterns of
// non-negative values order like the values; negative values and NaN have
// larger patterns and are rechecked exactly), so a packed 16-bit maximum
// decides; for thr < 0 (tb = -1) every run passes.  The words arrive as
// scalars: a bit cast of a vector element expression reads the vector's
// first element with this compiler.
__device__ __forceinline__ bool bf16x8_maybe_above(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                                   const PeakMarks &m) {
    const marks_u16x2_t x = __builtin_elementwise_max(
        __builtin_elementwise_max(__builtin_bit_cast(marks_u16x2_t, w0), __builtin_bit_cast(marks_u16x2_t, w1)),
        __builtin_elementwise_max(__builtin_bit_cast(marks_u16x2_t, w2), __builtin_bit_cast(marks_u16x2_t, w3)));
    return ((int32_t)x.x > m.tb) | ((int32_t)x.y > m.tb);
}

}  // namespace fdas
