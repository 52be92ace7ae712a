// Overlap-save correlation on the matrix cores: BF16 form, segment L = 4096.
//
// Same plane as the other kernels (Section "Detailed explanation": windows,
// transform, multiply by each template's transform, inverse transform, keep
// the central V = L - M outputs).  Every stage of every transform is a
// 16-point DFT on the matrix cores (16x16x32 bf16 MFMA, FP32 accumulation);
// factorisation and LDS layouts are in mfma4096.hpp.  One workgroup of 16
// waves owns a segment and a chunk of templates; wave w owns MFMA group
// Q = w of every stage:
//
//   forward  F1 (input rounded to bf16) -> LDS B -> F2 -> LDS A -> F3: the
//            segment spectrum X[k1, k2, k3] ends in registers in the first
//            inverse stage's B-operand layout, kept as (Re, -Im) and (Im, Re)
//            bf16 pairs so each product with a template value is two
//            v_dot2_f32_bf16.
//   template j: the bank entry of j + 1 is prefetched and its product with
//            X formed after I2 of template j; Y = X * H_j -> I1 ->
//            LDS A -> barrier -> (flush of template j - 1's row) -> I2 ->
//            LDS B -> barrier -> I3.  All three inverse stages run with the
//            operands swapped (transposed outputs): each lane then holds four
//            consecutive values of the next stage's K digit, so every
//            exchange is one 16-byte LDS write and one 16-byte read, and I3
//            leaves four consecutive time samples per lane -> |y|^2 staged in
//            LDS in the plane's type, written to the plane one barrier later
//            with coalesced vector stores.
// All twiddles live in the per-group stage operators, so the vector ALU only
// forms the template product, packs stage outputs to bf16 and squares.
// Register use stays at 64 VGPRs or fewer, so two workgroups (eight waves per
// SIMD) share a CU.
// A marking instance (kMark) also sets the peak finder's tile flags for the
// cells it stores above a threshold, so a fused peak search need not read
// the plane back to find the tiles worth examining.
#include "fft_valu.hpp"
#include "internal.hpp"
#include "marks.hpp"
#include "mfma4096.hpp"
#include "plane_io.hpp"

#include <algorithm>

namespace fdas {
namespace m4k {

constexpr int kWv = 16;           // waves per workgroup
constexpr int kThr = 64 * kWv;
constexpr int kGpw = 16 / kWv;    // MFMA groups (of 16 columns) per wave and stage
constexpr int kWavesPerEU = 8;    // two workgroups per CU

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

struct alignas(16) Op {
    uint32_t w[4];
};

__device__ __forceinline__ f32x4_t mma(const Op &a, const Op &b) {
    const f32x4_t z = {0.f, 0.f, 0.f, 0.f};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), z,
                                                   0, 0, 0);
}

typedef float f32x2_t __attribute__((ext_vector_type(2)));

// a.lo * b.lo + a.hi * b.hi of two bf16 pairs plus c, in FP32
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c, false);
}

// Two FP32 zeros in one 64-bit register pair (one 64-bit move instead of two
// 32-bit ones for the accumulators of v_dot2c; the empty asm emits nothing)
__device__ __forceinline__ f32x2_t zero_pair() {
    uint64_t z = 0;
    asm volatile("" : "+v"(z));
    return __builtin_bit_cast(f32x2_t, z);
}


__device__ __forceinline__ Op load_op(const uint32_t *tab, int op, int lane) {
    const uint4 v = reinterpret_cast<const uint4 *>(tab + op * kOpWords)[lane];
    return Op{{v.x, v.y, v.z, v.w}};
}

// Inverse-stage exchange: 16-byte chunks of four consecutive K values, chunk
// (a, b, g) at word 4 (256 g + 16 a + ((a + b) & 15)).  I1 writes with a fixed
// per wave and b = lane column, I2 reads with a = lane column and b fixed (and
// likewise I2 -> I3): the skew (a + b) & 15 spreads both patterns over all
// bank groups.
__device__ __forceinline__ int chunk_addr(int a, int b, int g) { return 4 * (256 * g + 16 * a + ((a + b) & 15)); }

// Staging of one template row's powers between I3 and the plane store.
// FP32 plane: one float per sample at t + 4 (t >> 8); BF16 plane: the bf16
// value, two samples per word, at word t / 2 + 4 (t >> 8), so runs of 8
// samples are 16-byte aligned for the flush reads.  The FP32 pad keeps the
// I3 writes (lanes 256 samples apart) and the flush reads conflict-free; the
// BF16 pad leaves a two-way conflict in the I3 writes (lanes c and c + 8),
// cheaper than the conflict of reading 8 samples as two 8-byte halves under
// a 2-word pad (measured).
template <class PT>
struct Stage;
template <>
struct Stage<float> {
    static constexpr int kWords = kL + 4 * 16;
    static __device__ __forceinline__ void put4(uint32_t *st, int t0, float a, float b, float c, float d) {
        *reinterpret_cast<float4 *>(&st[t0 + 4 * (t0 >> 8)]) = make_float4(a, b, c, d);
    }
    static __device__ __forceinline__ float4 chunk(const uint32_t *st, int t0) {
        return *reinterpret_cast<const float4 *>(&st[t0 + 4 * (t0 >> 8)]);
    }
    // samples t0 .. t0 + 3 -> plane, vector or element-wise; kMark: the
    // peak tiles of the kept samples flagged when one of the four is above
    // the threshold (plane row z, column seg0 + t).  kShift: when the row
    // starts sh floats past a 16-byte boundary (the same sh on every lane),
    // the thread stores the aligned run [t0 - sh, t0 - sh + 4) instead, from
    // its own staged chunk and the preceding one.
    template <bool kMark, bool kShift>
    static __device__ __forceinline__ void flush4(const uint32_t *st, int t0, float *row, bool vec, int lo, int hi,
                                                  const PeakMarks &m, int64_t z, int64_t seg0) {
        if constexpr (!kShift) {
            const float4 v = chunk(st, t0);
            const float vv[4] = {v.x, v.y, v.z, v.w};
            if (vec) {
                const f32x4_t u = {v.x, v.y, v.z, v.w};
                __builtin_nontemporal_store(u, reinterpret_cast<f32x4_t *>(row + t0));
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (t0 + i >= lo && t0 + i < hi) row[t0 + i] = vv[i];
            }
            if constexpr (kMark) {
                if ((vv[0] > m.thr) | (vv[1] > m.thr) | (vv[2] > m.thr) | (vv[3] > m.thr)) {   // rare
                    // an opaque copy keeps the run bounds (loop-invariant per
                    // lane) from being hoisted and held across the template loop
                    int t = t0;
                    asm volatile("" : "+v"(t));
                    mark_run(m, (uint32_t)z * (uint32_t)m.n_cb, (int32_t)seg0, max(t, lo), min(t + 3, hi - 1));
                }
            }
            return;
        }
        const int sh = (int)((reinterpret_cast<uintptr_t>(row) >> 2) & 3);
        float4 v = chunk(st, t0);
        int t = t0;
        if (sh != 0) {
            // t0 = 0: the samples before it are outside every row's kept range
            const float4 p = chunk(st, max(t0 - 4, 0));
            v = sh == 1 ? make_float4(p.w, v.x, v.y, v.z)
                        : (sh == 2 ? make_float4(p.z, p.w, v.x, v.y) : make_float4(p.y, p.z, p.w, v.x));
            t = t0 - sh;
        }
        const float vv[4] = {v.x, v.y, v.z, v.w};
        if (t >= lo && t + 4 <= hi) {
            const f32x4_t u = {v.x, v.y, v.z, v.w};
            __builtin_nontemporal_store(u, reinterpret_cast<f32x4_t *>(row + t));
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (t + i >= lo && t + i < hi) row[t + i] = vv[i];
        }
        if constexpr (kMark) {
            if ((vv[0] > m.thr) | (vv[1] > m.thr) | (vv[2] > m.thr) | (vv[3] > m.thr)) {   // rare
                asm volatile("" : "+v"(t));   // opaque copy, as above
                mark_run(m, (uint32_t)z * (uint32_t)m.n_cb, (int32_t)seg0, max(t, lo), min(t + 3, hi - 1));
            }
        }
        // Shifted runs cover samples [-sh, kL - sh).  With fewer than 8 taps
        // the kept samples reach past kL - sh: thread 0 stores that tail.
        if (sh != 0 && t0 == 0 && hi > kL - sh) {
            const float4 q = chunk(st, kL - 4);
            const float qq[4] = {q.x, q.y, q.z, q.w};
            bool above = false;
            for (int i = 4 - sh; i < 4 && kL - 4 + i < hi; ++i) {
                row[kL - 4 + i] = qq[i];
                above |= qq[i] > m.thr;
            }
            if constexpr (kMark) {
                if (above) mark_run(m, (uint32_t)z * (uint32_t)m.n_cb, (int32_t)seg0, kL - sh, hi - 1);
            }
        }
    }
};
// Eight bf16 samples starting S (1..7) samples before the run held in c,
// from the words of the preceding run p and of c (two samples per word,
// lower half first).
template <int S>
__device__ __forceinline__ uint4 bf16_run_back(const uint4 &p, const uint4 &c) {
    const uint32_t w[8] = {p.x, p.y, p.z, p.w, c.x, c.y, c.z, c.w};
    constexpr int b = 4 - S / 2;
    uint32_t o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if constexpr (S & 1)
            o[i] = __builtin_amdgcn_alignbit(w[b + i], w[b - 1 + i], 16);   // upper half of one word, lower of the next
        else
            o[i] = w[b + i];
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

template <>
struct Stage<__bf16> {
    static constexpr int kWords = kL / 2 + 4 * 16;
    static __device__ __forceinline__ void put4(uint32_t *st, int t0, float a, float b, float c, float d) {
        uint2 u;
        u.x = bf16_pack(a, b);
        u.y = bf16_pack(c, d);
        *reinterpret_cast<uint2 *>(&st[t0 / 2 + 4 * (t0 >> 8)]) = u;
    }
    static __device__ __forceinline__ uint4 run(const uint32_t *st, int t0) {
        return *reinterpret_cast<const uint4 *>(&st[t0 / 2 + 4 * (t0 >> 8)]);
    }
    // Eight samples per lane (t0 a multiple of 8), one 16-byte store.
    // !kShift (launches whose rows all start on 16-byte boundaries): vec8
    // says whether the run [t0, t0 + 8) is stored whole.  kShift: when the
    // row starts sh samples past a 16-byte boundary (sh is the same for
    // every lane of the workgroup), the lane stores the aligned run of
    // samples [t0 - sh, t0 - sh + 8) instead, assembled from its own staged
    // run and the preceding one, so rows of any length keep 16-byte stores;
    // vmask bit k: the run [t0 - k, t0 - k + 8) lies inside the kept samples
    // [lo, hi).  Runs not stored whole are stored element by element.
    // kMark: as for FP32, when the packed prefilter passes.
    template <bool kMark, bool kShift>
    static __device__ __forceinline__ void flush8(const uint32_t *st, int t0, __bf16 *row, bool vec8, uint32_t vmask,
                                                  int lo, int hi, const PeakMarks &m, int64_t z, int64_t seg0) {
        if constexpr (!kShift) {
            const uint4 u = run(st, t0);
            if (vec8) {
                const u32x4_t w = {u.x, u.y, u.z, u.w};
                __builtin_nontemporal_store(w, reinterpret_cast<u32x4_t *>(row + t0));
            } else {
                const uint32_t ww[4] = {u.x, u.y, u.z, u.w};
                uint16_t *r16 = reinterpret_cast<uint16_t *>(row);
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (t0 + i >= lo && t0 + i < hi) r16[t0 + i] = (uint16_t)(ww[i >> 1] >> (16 * (i & 1)));
            }
            if constexpr (kMark) {
                const uint32_t w0 = u.x, w1 = u.y, w2 = u.z, w3 = u.w;
                if (bf16x8_maybe_above(w0, w1, w2, w3, m)) {   // rare
                    int t = t0;   // opaque copy, as for FP32
                    asm volatile("" : "+v"(t));
                    mark_run(m, (uint32_t)z * (uint32_t)m.n_cb, (int32_t)seg0, max(t, lo), min(t + 7, hi - 1));
                }
            }
            return;
        }
        const int sh = (int)((reinterpret_cast<uintptr_t>(row) >> 1) & 7);
        uint4 u = run(st, t0);
        int t = t0;
        if (sh != 0) {
            // t0 = 0: the samples before it are outside every row's kept range
            const uint4 p = run(st, max(t0 - 8, 0));
            switch (sh) {
                case 1: u = bf16_run_back<1>(p, u); break;
                case 2: u = bf16_run_back<2>(p, u); break;
                case 3: u = bf16_run_back<3>(p, u); break;
                case 4: u = bf16_run_back<4>(p, u); break;
                case 5: u = bf16_run_back<5>(p, u); break;
                case 6: u = bf16_run_back<6>(p, u); break;
                default: u = bf16_run_back<7>(p, u); break;
            }
            t = t0 - sh;
        }
        if ((vmask >> sh) & 1) {
            const u32x4_t w = {u.x, u.y, u.z, u.w};
            __builtin_nontemporal_store(w, reinterpret_cast<u32x4_t *>(row + t));
        } else {
            // the kept samples [pa, pb) of the (16-byte aligned) run: whole
            // words as 4-byte stores, an odd sample at either end alone
            const uint32_t ww[4] = {u.x, u.y, u.z, u.w};
            const int pa = min(max(lo - t, 0), 8), pb = min(max(hi - t, 0), 8);
            uint16_t *r16 = reinterpret_cast<uint16_t *>(row + t);
            uint32_t *r32 = reinterpret_cast<uint32_t *>(row + t);
            if ((pa & 1) && pa < pb) r16[pa] = (uint16_t)(ww[pa >> 1] >> 16);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (2 * i >= pa && 2 * i + 2 <= pb) r32[i] = ww[i];
            if ((pb & 1) && pb - 1 >= pa) r16[pb - 1] = (uint16_t)ww[(pb - 1) >> 1];
        }
        if constexpr (kMark) {
            const uint32_t w0 = u.x, w1 = u.y, w2 = u.z, w3 = u.w;
            if (bf16x8_maybe_above(w0, w1, w2, w3, m)) {   // rare
                asm volatile("" : "+v"(t));   // opaque copy, as for FP32
                mark_run(m, (uint32_t)z * (uint32_t)m.n_cb, (int32_t)seg0, max(t, lo), min(t + 7, hi - 1));
            }
        }
        // Shifted runs cover samples [-sh, kL - sh).  With fewer than 16 taps
        // the kept samples reach past kL - sh: lane 0 stores that tail.
        if (sh != 0 && t0 == 0 && hi > kL - sh) {
            const uint4 q = run(st, kL - 8);
            const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
            uint16_t *r16 = reinterpret_cast<uint16_t *>(row);
            for (int i = 8 - sh; i < 8 && kL - 8 + i < hi; ++i) r16[kL - 8 + i] = (uint16_t)(qq[i >> 1] >> (16 * (i & 1)));
            if constexpr (kMark) {
                if (bf16x8_maybe_above(q.x, q.y, q.z, q.w, m))
                    mark_run(m, (uint32_t)z * (uint32_t)m.n_cb, (int32_t)seg0, kL - sh, hi - 1);
            }
        }
    }
};

// Per-thread flush plan.  FP32 rows: thread tid owns time samples
// [t0, t0 + 4) with t0 = 4 (tid + h kThr), h < kFlushChunks (consecutive
// lanes take consecutive chunks).  BF16 rows: the threads of one half of the
// workgroup own 8 samples each, t0 = 8 (tid mod 512), so every store is 16
// bytes (1 KB per wave); the halves take even and odd templates in turn.
// vec[h] / vec8: the chunk is entirely kept, inside the plane and aligned
// for one vector store in every template row; vmask8: the same for the BF16
// run shifted back by k samples (bit k, see Stage<__bf16>::flush8).  Samples
// [lo, hi) of a row are kept.
constexpr int kFlushChunks = kL / (4 * kThr);
struct FlushPlan {
    bool vec[kFlushChunks];
    bool vec8;
    uint32_t vmask8;
    int t08;             // BF16 run of this thread (shifting instance)
    int lo, hi;
};

template <class PT, bool kShift>
__device__ __forceinline__ FlushPlan flush_plan(const PT *plane, int64_t seg0, int64_t n, int half, int tid) {
    FlushPlan f;
    constexpr uintptr_t kChunkBytes = 4 * sizeof(PT);   // 4 elements: 8 B (bf16) or 16 B (fp32)
    const bool rows_aligned = (n % 4) == 0;             // every row start keeps the chunk alignment
    f.lo = half;
    f.hi = (int)min((int64_t)(kL - half), n - seg0);    // columns >= n are outside the plane
#pragma unroll
    for (int h = 0; h < kFlushChunks; ++h) {
        const int t0 = 4 * (tid + h * kThr);
        f.vec[h] = rows_aligned && (reinterpret_cast<uintptr_t>(plane + seg0 + t0) % kChunkBytes) == 0 &&
                   t0 >= f.lo && t0 + 4 <= f.hi;
    }
    {
        // The shifting instance rotates the runs over the threads of a half
        // so that the run holding the first kept sample sits at lane 62 or 63
        // of the first wave: with V >= 8 * 449 the run holding the last kept
        // sample (and the tail of fewer than 16 taps) falls in that wave too,
        // so one wave per row, not two, stores the partial runs.
        const int t0 = kShift ? 8 * (((tid & 511) + ((f.lo >> 3) - 62)) & 511) : 8 * (tid & 511);
        f.t08 = t0;
        f.vec8 = (n % 8) == 0 && (reinterpret_cast<uintptr_t>(plane + seg0 + t0) % 16) == 0 && t0 >= f.lo &&
                 t0 + 8 <= f.hi;
        uint32_t vm = 0;
        if constexpr (kShift) {
#pragma unroll
            for (int k = 0; k < 8; ++k) vm |= (uint32_t)(t0 - k >= f.lo && t0 - k + 8 <= f.hi) << k;
        }
        f.vmask8 = vm;
    }
    return f;
}

// Row z of the plane (its segment starts at column seg0) from the staging
// buffer; kMark: with its peak tiles marked.
template <class PT, bool kMark, bool kShift>
__device__ __forceinline__ void flush(const uint32_t *stage, PT *row_seg, const FlushPlan &f, int tid, int jpar,
                                      const PeakMarks &m, int64_t z, int64_t seg0) {
    if constexpr (sizeof(PT) == 2) {
        // lower half of the workgroup: even templates, upper half: odd ones
        if ((tid >> 9) == jpar)
            Stage<PT>::template flush8<kMark, kShift>(stage, kShift ? f.t08 : 8 * (tid & 511), row_seg, f.vec8, f.vmask8, f.lo, f.hi, m,
                                                        z, seg0);
    } else {
#pragma unroll
        for (int h = 0; h < kFlushChunks; ++h) {
            const int t0 = 4 * (tid + h * kThr);
            Stage<PT>::template flush4<kMark, kShift>(stage, t0, row_seg, f.vec[h], f.lo, f.hi, m, z, seg0);
        }
    }
}

// One tile: segment s of the spectrum (n bins) against templates [j0, j1),
// writing plane rows j0 .. j1 - 1 (row stride n); kMark: marking the peak
// tiles (m) of the cells it stores above the threshold; kShift: rows may
// start anywhere (see Stage<>::flush8 and flush4).  Called by the whole
// workgroup; contains barriers.
template <class PT, bool kOpaqueLane = false, bool kMark = false, bool kShift = false>
__device__ __forceinline__ void m4k_tile(const float2 *__restrict__ spec, int64_t n, const uint32_t *__restrict__ bank,
                                         const uint32_t *__restrict__ tab, PT *__restrict__ plane, int32_t M,
                                         int32_t V, int64_t s, int j0, int j1, uint32_t *bufA, uint32_t *bufB,
                                         uint32_t *stage, const PeakMarks &m) {
    int tid = (int)threadIdx.x, w = tid >> 6, lane = tid & 63;
    if constexpr (kOpaqueLane) {
        // per-tile copies the compiler cannot prove loop-invariant, so that a
        // persistent caller does not keep every lane address live across tiles
        w = __builtin_amdgcn_readfirstlane(w);
        asm volatile("" : "+s"(w));
        asm volatile("" : "+v"(lane));
        tid = 64 * w + lane;
    }
    const int c = lane & 15, g = lane >> 4;
    const int half = M / 2;
    const int64_t seg0 = s * (int64_t)V - half;   // plane column of time index t is seg0 + t
    // ---------------- forward transform ----------------
    // F1: n2 = Q, column n3 = c, K: n1 = 4 g + p  ->  rows k1 = 4 g + e  -> buffer B
    const bool inside = seg0 >= 0 && seg0 + kL <= n;   // no window sample falls outside [0, n)
    const float2 *win = spec + seg0;
#pragma unroll
    for (int q = 0; q < kGpw; ++q) {
        const int Q = kGpw * w + q;
        Op b;
        float2 v[4];
        if (inside) {
#pragma unroll
            for (int p = 0; p < 4; ++p) v[p] = win[256 * (4 * g + p) + 16 * Q + c];
        } else {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int64_t idx = seg0 + 256 * (4 * g + p) + 16 * Q + c;
                v[p] = (idx >= 0 && idx < n) ? spec[idx] : make_float2(0.f, 0.f);
            }
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) b.w[p] = bf16_pack(v[p].x, v[p].y);
        const f32x4_t dre = mma(load_op(tab, OP_F12 + 2 * Q, lane), b);
        const f32x4_t dim = mma(load_op(tab, OP_F12 + 2 * Q + 1, lane), b);
        uint4 o;
        o.x = bf16_pack(dre[0], dim[0]);
        o.y = bf16_pack(dre[1], dim[1]);
        o.z = bf16_pack(dre[2], dim[2]);
        o.w = bf16_pack(dre[3], dim[3]);
        *reinterpret_cast<uint4 *>(&bufB[addrB(4 * g, Q, c)]) = o;   // 4 consecutive k1
    }
    __syncthreads();
    // F2: n3 = Q, column k1 = c, K: n2 = 4 g + p  ->  rows k2 = 4 g + e  -> buffer A
#pragma unroll
    for (int q = 0; q < kGpw; ++q) {
        const int Q = kGpw * w + q;
        Op b;
#pragma unroll
        for (int p = 0; p < 4; ++p) b.w[p] = bufB[addrB(c, 4 * g + p, Q)];
        const f32x4_t dre = mma(load_op(tab, OP_F12 + 2 * Q, lane), b);
        const f32x4_t dim = mma(load_op(tab, OP_F12 + 2 * Q + 1, lane), b);
        uint4 o;
        o.x = bf16_pack(dre[0], dim[0]);
        o.y = bf16_pack(dre[1], dim[1]);
        o.z = bf16_pack(dre[2], dim[2]);
        o.w = bf16_pack(dre[3], dim[3]);
        *reinterpret_cast<uint4 *>(&bufA[addrA(c, 4 * g, Q)]) = o;   // 4 consecutive k2
    }
    __syncthreads();
    // F3: k1 = Q, column k2 = c, K: n3 = 4 g + p -> X[Q, c, 4 g + e] in registers.
    // Each wave reads exactly the buffer-A words its own I1 writes later, so
    // no barrier is needed before the template loop.
    uint32_t sA[kGpw][4], sB[kGpw][4];
#pragma unroll
    for (int q = 0; q < kGpw; ++q) {
        const int Q = kGpw * w + q;
        Op b;
#pragma unroll
        for (int p = 0; p < 4; ++p) b.w[p] = bufA[addrA(Q, c, 4 * g + p)];
        const f32x4_t dre = mma(load_op(tab, OP_F3 + 2 * Q, lane), b);
        const f32x4_t dim = mma(load_op(tab, OP_F3 + 2 * Q + 1, lane), b);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            sA[q][p] = bf16_pack(dre[p], -dim[p]);
            sB[q][p] = bf16_pack(dim[p], dre[p]);
        }
    }

    // ---------------- per-group inverse operators ----------------
    Op a1re[kGpw], a1im[kGpw], a23re[kGpw], a23im[kGpw];
#pragma unroll
    for (int q = 0; q < kGpw; ++q) {
        const int Q = kGpw * w + q;
        a1re[q] = load_op(tab, OP_I1 + 2 * Q, lane);
        a1im[q] = load_op(tab, OP_I1 + 2 * Q + 1, lane);
        a23re[q] = load_op(tab, OP_I23 + 2 * Q, lane);
        a23im[q] = load_op(tab, OP_I23 + 2 * Q + 1, lane);
    }

    const FlushPlan fp = flush_plan<PT, kShift>(plane, seg0, n, half, tid);
    const uint4 *bank4 = reinterpret_cast<const uint4 *>(bank) + (kGpw * w) * 64 + lane;

    // One template: I1 (group k1 = Q) on X * H_j, I2 (group n3), I3 (group n2).
    // template product Y = X * H_j into the I1 operand (kept in bin[])
    Op bin[kGpw];
    auto product = [&](const uint4 (&hc)[kGpw]) {
#pragma unroll
        for (int q = 0; q < kGpw; ++q) {
            const uint32_t hw[4] = {hc[q].x, hc[q].y, hc[q].z, hc[q].w};
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const f32x2_t z = zero_pair();
                bin[q].w[p] = bf16_pack(dot2(sA[q][p], hw[p], z.x), dot2(sB[q][p], hw[p], z.y));
            }
        }
    };

    // One template.  Single-segment launches form the product of the next
    // template (bank entry hn) between I2 and the second barrier, which
    // balances the vector-ALU work of the two barrier intervals (template j's
    // product is then already in bin[]); the persistent batch kernel forms
    // template j's product (bank entry hc) just before its I1, which needs
    // fewer registers live across the barriers.
    auto one_template = [&](int j, const uint4 (&hc)[kGpw], const uint4 (&hn)[kGpw], bool has_next) {
        if constexpr (kOpaqueLane) product(hc);
        // I1: DFT16 over k3 with e(n3 k1), transposed: lane (c, g) receives
        // n3 = c, k2 = 4 g + e -> one 16-byte chunk of buffer A
#pragma unroll
        for (int q = 0; q < kGpw; ++q) {
            const int Q = kGpw * w + q;
            const f32x4_t dre = mma(bin[q], a1re[q]), dim = mma(bin[q], a1im[q]);
            uint4 o;
            o.x = bf16_pack(dre[0], dim[0]);
            o.y = bf16_pack(dre[1], dim[1]);
            o.z = bf16_pack(dre[2], dim[2]);
            o.w = bf16_pack(dre[3], dim[3]);
            *reinterpret_cast<uint4 *>(&bufA[chunk_addr(Q, c, g)]) = o;   // (k1, n3, k2 block)
        }
        __syncthreads();
        if (j > j0) flush<PT, kMark, kShift>(stage, plane + (int64_t)(j - 1) * n + seg0, fp, tid, (j - 1) & 1, m, j - 1, seg0);
        // I2: DFT16 over k2 with e(16 n3 k2), transposed: lane (c, g)
        // receives n2 = c, k1 = 4 g + e -> one 16-byte chunk of buffer B
#pragma unroll
        for (int q = 0; q < kGpw; ++q) {
            const int Q = kGpw * w + q;
            const uint4 v = *reinterpret_cast<const uint4 *>(&bufA[chunk_addr(c, Q, g)]);   // k1 = c, n3 = Q
            const Op b = {{v.x, v.y, v.z, v.w}};
            const f32x4_t dre = mma(b, a23re[q]), dim = mma(b, a23im[q]);
            uint4 o;
            o.x = bf16_pack(dre[0], dim[0]);
            o.y = bf16_pack(dre[1], dim[1]);
            o.z = bf16_pack(dre[2], dim[2]);
            o.w = bf16_pack(dre[3], dim[3]);
            *reinterpret_cast<uint4 *>(&bufB[chunk_addr(c, Q, g)]) = o;   // (n2, n3, k1 block)
        }
        if constexpr (!kOpaqueLane) {
            if (has_next) product(hn);
        }
        __syncthreads();
        // I3: DFT16 over k1 with e(16 n2 k1); rows n1 = 4 g + e; |y|^2 -> staging
#pragma unroll
        for (int q = 0; q < kGpw; ++q) {
            const int Q = kGpw * w + q;
            const uint4 v = *reinterpret_cast<const uint4 *>(&bufB[chunk_addr(Q, c, g)]);   // n2 = Q, n3 = c
            const Op b = {{v.x, v.y, v.z, v.w}};
            const f32x4_t dre = mma(b, a23re[q]), dim = mma(b, a23im[q]);
            Stage<PT>::put4(stage, 256 * c + 16 * Q + 4 * g, dre[0] * dre[0] + dim[0] * dim[0],
                            dre[1] * dre[1] + dim[1] * dim[1], dre[2] * dre[2] + dim[2] * dim[2],
                            dre[3] * dre[3] + dim[3] * dim[3]);
        }
    };

    // the inverse stages use the chunk layout: every wave must be done with
    // its forward reads of buffer A
    __syncthreads();
    // bank entries in two statically assigned register sets: the entry of
    // template j + 1 is loaded while template j runs
    uint4 hA[kGpw], hB[kGpw];
#pragma unroll
    for (int q = 0; q < kGpw; ++q) hA[q] = bank4[(size_t)j0 * (kL / 4) + q * 64];
    if constexpr (!kOpaqueLane) product(hA);
    for (int j = j0; j < j1; j += 2) {
        if (j + 1 < j1) {
#pragma unroll
            for (int q = 0; q < kGpw; ++q) hB[q] = bank4[(size_t)(j + 1) * (kL / 4) + q * 64];
        }
        one_template(j, hA, hB, j + 1 < j1);
        if (j + 1 >= j1) break;
        if (j + 2 < j1) {
#pragma unroll
            for (int q = 0; q < kGpw; ++q) hA[q] = bank4[(size_t)(j + 2) * (kL / 4) + q * 64];
        }
        one_template(j + 1, hB, hA, j + 2 < j1);
    }
    __syncthreads();
    flush<PT, kMark, kShift>(stage, plane + (int64_t)(j1 - 1) * n + seg0, fp, tid, (j1 - 1) & 1, m, j1 - 1, seg0);
}

#define M4K_ATTR __attribute__((amdgpu_flat_work_group_size(kThr, kThr), amdgpu_waves_per_eu(kWavesPerEU)))

// One spectrum: workgroup b takes template chunk b mod n_chunks of segment
// b / n_chunks.  kMark: the peak tiles of the plane (m) are marked as well;
// kShift: some row starts are not 16-byte aligned.
template <class PT, bool kMark, bool kShift>
__global__ void M4K_ATTR correlate_mfma4096(const float2 *__restrict__ spec, int64_t n,
                                            const uint32_t *__restrict__ bank, const uint32_t *__restrict__ tab,
                                            PT *__restrict__ plane, int32_t M, int32_t V, int32_t n_z,
                                            int32_t z_chunk, int32_t n_chunks, PeakMarks m) {
    __shared__ __align__(16) uint32_t bufA[kBufWords];
    __shared__ __align__(16) uint32_t bufB[kBufWords];
    __shared__ __align__(16) uint32_t stage[Stage<PT>::kWords];
    const int chunk = blockIdx.x % n_chunks;
    const int64_t s = blockIdx.x / n_chunks;
    const int j0 = chunk * z_chunk;
    const int j1 = min(j0 + z_chunk, n_z);
    if (j0 >= j1) return;
    m4k_tile<PT, false, kMark, kShift>(spec, n, bank, tab, plane, M, V, s, j0, j1, bufA, bufB, stage, m);
}

// Many spectra in one persistent launch.  Tiles are (job, segment, template
// chunk); each chunk has its own queue of segments (all jobs' segments in
// order, job by binary search over the segment prefix seg_base).  Workgroups
// are dispatched round-robin over the eight XCDs, so a workgroup starts on
// chunk (XCD mod n_chunks): each XCD's L2 then holds only its chunks' part of
// the template bank.  A workgroup whose queue is empty moves on to the next
// chunk's queue, so ragged lengths still balance across the CUs.  kMark:
// the peak tiles of every job's plane are marked as well (m.flags and
// m.cflags are the batch's arrays, each job's part at its tile_base and
// chunk_base).  kShift: as for one spectrum.
constexpr int kXcds = 8;

template <class PT, bool kMark, bool kShift>
__global__ void M4K_ATTR correlate_mfma4096_batch(const float2 *__restrict__ spectra,
                                                  const fdas_batch_job *__restrict__ jobs, int32_t n_jobs,
                                                  int32_t n_segs, int32_t *__restrict__ counters,
                                                  const uint32_t *__restrict__ bank, const uint32_t *__restrict__ tab,
                                                  PT *__restrict__ planes, int32_t M, int32_t V, int32_t n_z,
                                                  int32_t z_chunk, int32_t n_chunks, PeakMarks m) {
    __shared__ __align__(16) uint32_t bufA[kBufWords];
    __shared__ __align__(16) uint32_t bufB[kBufWords];
    __shared__ __align__(16) uint32_t stage[Stage<PT>::kWords];
    __shared__ int s_chunk, s_seg;
    const int c0 = (int)(blockIdx.x % kXcds) % n_chunks;
    int c_off = 0;   // used by thread 0 only
    for (;;) {
        if (threadIdx.x == 0) {
            int sg = n_segs;
            while (c_off < n_chunks) {
                sg = atomicAdd(&counters[(c0 + c_off) % n_chunks], 1);
                if (sg < n_segs) break;
                ++c_off;
            }
            s_chunk = c_off < n_chunks ? (c0 + c_off) % n_chunks : -1;
            s_seg = sg;
        }
        __syncthreads();
        // the tile and everything derived from it are the same on every lane:
        // keep them in scalar registers
        const int chunk = __builtin_amdgcn_readfirstlane(s_chunk);
        if (chunk < 0) return;                    // uniform: every wave leaves together
        const int sg = __builtin_amdgcn_readfirstlane(s_seg);
        int lo = 0, hi = n_jobs - 1;              // last job with seg_base <= sg
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].seg_base <= sg) lo = mid;
            else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const int64_t spec_off = jobs[lo].spec_off, nb = jobs[lo].n_bins;
        const int64_t plane_off = jobs[lo].plane_off;
        const int s = sg - (int)jobs[lo].seg_base;
        const int j0 = chunk * z_chunk;
        const int j1 = min(j0 + z_chunk, n_z);
        // an opaque zero keeps the per-tile operator loads inside the loop, so
        // they are not hoisted out and held in registers across tiles
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        PeakMarks mj = m;
        if constexpr (kMark) {
            mj.flags = m.flags + jobs[lo].tile_base;
            mj.cflags = m.cflags + jobs[lo].chunk_base;
            mj.n_cb = (int32_t)((nb + kPeakTileCols - 1) / kPeakTileCols);
        }
        m4k_tile<PT, true, kMark, kShift>(spectra + spec_off + opaque, nb, bank + opaque, tab + opaque,
                                  planes + plane_off + opaque, M, V + opaque, s, j0, j1, bufA, bufB, stage, mj);
    }
}

namespace {
// Do the rows start on 16-byte boundaries in every segment?  Row z of the
// segment at column s V - M / 2 starts at element plane_off + z n + s V - M / 2.
template <class PT>
bool rows_aligned(const fdas_plan_s &p, const void *plane, int64_t plane_off, int64_t n) {
    constexpr int64_t e = 16 / sizeof(PT);   // elements per 16 bytes
    return (reinterpret_cast<uintptr_t>(plane) % 16) == 0 && plane_off % e == 0 && n % e == 0 && p.V % e == 0 &&
           (p.M / 2) % e == 0;
}

template <class PT, bool kMark>
hipError_t launch(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, const PeakMarks &m,
                  hipStream_t st) {
    const int64_t n_seg = (n + p.V - 1) / p.V;
    const int64_t blocks = n_seg * p.n_chunks;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const auto *ws = static_cast<const unsigned char *>(p.ws);
    auto kernel = rows_aligned<PT>(p, plane, 0, n) ? correlate_mfma4096<PT, kMark, false>
                                                   : correlate_mfma4096<PT, kMark, true>;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kThr), 0, st,
                       static_cast<const float2 *>(spec), n, reinterpret_cast<const uint32_t *>(ws + p.off_bank),
                       reinterpret_cast<const uint32_t *>(ws + p.off_tab), static_cast<PT *>(plane), p.M, p.V,
                       p.cfg.n_z, p.z_chunk, p.n_chunks, m);
    return hipGetLastError();
}
template <class PT, bool kMark>
hipError_t launch_batch(const fdas_plan_s &p, const void *spectra, void *planes, const PeakMarks &m,
                        hipStream_t st) {
    auto *ws = static_cast<unsigned char *>(p.ws);
    int32_t *counters = reinterpret_cast<int32_t *>(ws + p.off_batch);
    const auto *jobs = reinterpret_cast<const fdas_batch_job *>(ws + p.off_batch + p.batch_hdr);
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, st, counters, p.n_chunks);
    int dev = 0, cus = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t grid = std::min<int64_t>((int64_t)cus * 2, std::max<int64_t>(p.batch_tiles, 1));
    bool aligned = true;
    for (const fdas_batch_job &j : p.batch_host)
        aligned = aligned && rows_aligned<PT>(p, planes, j.plane_off, j.n_bins);
    auto kernel = aligned ? correlate_mfma4096_batch<PT, kMark, false> : correlate_mfma4096_batch<PT, kMark, true>;
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(kThr), 0, st,
                       static_cast<const float2 *>(spectra), jobs, p.batch_jobs,
                       (int32_t)(p.batch_tiles / p.n_chunks), counters,
                       reinterpret_cast<const uint32_t *>(ws + p.off_bank),
                       reinterpret_cast<const uint32_t *>(ws + p.off_tab), static_cast<PT *>(planes), p.M, p.V,
                       p.cfg.n_z, p.z_chunk, p.n_chunks, m);
    return hipGetLastError();
}

}  // namespace

}  // namespace m4k

hipError_t launch_correlate_m4k_batch(const fdas_plan_s &p, const void *spectra, void *planes, hipStream_t st) {
    if (p.L != m4k::kL || p.cfg.compute != FDAS_BF16) return hipErrorInvalidValue;
    const PeakMarks none{};
    if (p.cfg.plane_dtype == FDAS_BF16) return m4k::launch_batch<__bf16, false>(p, spectra, planes, none, st);
    if (p.cfg.plane_dtype == FDAS_FP32) return m4k::launch_batch<float, false>(p, spectra, planes, none, st);
    return hipErrorInvalidValue;
}

hipError_t launch_correlate_m4k_batch_marked(const fdas_plan_s &p, const void *spectra, void *planes,
                                             const PeakMarks &marks, hipStream_t st) {
    if (p.L != m4k::kL || p.cfg.compute != FDAS_BF16) return hipErrorInvalidValue;
    if (p.cfg.plane_dtype == FDAS_BF16) return m4k::launch_batch<__bf16, true>(p, spectra, planes, marks, st);
    if (p.cfg.plane_dtype == FDAS_FP32) return m4k::launch_batch<float, true>(p, spectra, planes, marks, st);
    return hipErrorInvalidValue;
}

hipError_t launch_correlate_m4k(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    if (p.L != m4k::kL || p.cfg.compute != FDAS_BF16) return hipErrorInvalidValue;
    const PeakMarks none{};
    if (p.cfg.plane_dtype == FDAS_BF16) return m4k::launch<__bf16, false>(p, spec, n, plane, none, st);
    if (p.cfg.plane_dtype == FDAS_FP32) return m4k::launch<float, false>(p, spec, n, plane, none, st);
    return hipErrorInvalidValue;
}

hipError_t launch_correlate_m4k_marked(const fdas_plan_s &p, const void *spec, int64_t n, void *plane,
                                       const PeakMarks &marks, hipStream_t st) {
    if (p.L != m4k::kL || p.cfg.compute != FDAS_BF16) return hipErrorInvalidValue;
    if (p.cfg.plane_dtype == FDAS_BF16) return m4k::launch<__bf16, true>(p, spec, n, plane, marks, st);
    if (p.cfg.plane_dtype == FDAS_FP32) return m4k::launch<float, true>(p, spec, n, plane, marks, st);
    return hipErrorInvalidValue;
}

}  // namespace fdas
