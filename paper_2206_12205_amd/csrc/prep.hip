// Spectrum preparation upstream of the correlation: single-precision real
// FFT, Nyquist dropped, DC zeroed, median-power normalisation.
//
// The paper keeps the real FFT that makes the spectrum in single precision
// (Section "Casting between single-precision and bfloat16") and the search
// takes the spectrum normalised so that noise powers are Exp(1):
//   X[k] = sum_t x[t] exp(-2 pi i k t / N_t), k in [0, N_t / 2),  X[0] = 0,
//   X[k] /= sqrt(median_{k >= 1} |X[k]|^2 / ln 2).
//
// Transform.  The N_t real samples read as N = N_t / 2 complex values
// z[m] = x[2m] + i x[2m+1] (the series reinterpreted, no copy).  The complex
// FFT of length N = N1 N2 (N1, N2 of the form 2^a or 3 * 2^a, at most 4096)
// runs as a four-step transform whose sub-transforms live in LDS:
//   n = N2 n1 + n2,  k = k1 + N1 k2,
//   Z[k] = sum_n2 e(-n2 k2 / N2) [ e(-n2 k1 / N) sum_n1 z[N2 n1 + n2] e(-n1 k1 / N1) ]
// (e(x) = exp(2 pi i x)).  Pass 1 (k_cols): a workgroup loads a few
// consecutive columns n2 (all n1), runs their length-N1 FFTs as Stockham
// passes in LDS (radix 16, 8, 4, 2 and one radix-3 pass), applies
// e(-n2 k1 / N) and writes Y[k1][n2].  Pass 2 (k_rows): a workgroup loads four
// consecutive rows k1 and the four rows N1 - k1 that hold the mirrored bins
// N - k, runs their length-N2 FFTs in LDS and forms the real spectrum
//   X[k] = (Z[k] + conj Z[N-k]) / 2 - i e(-k / 2N) (Z[k] - conj Z[N-k]) / 2,
// X[0] = 0.  Stage twiddles come from single-precision sincospi of exact
// integer ratios (their powers by complex products); every value passes
// log2 N radix stages.
//
// Median.  Exact selection of the middle power among the N - 1 bins k >= 1
// (an odd count, N even), by the powers' bit patterns (non-negative floats
// order like their patterns) in three rounds of 12, 10 and 10 bits: the first
// row pass stores the patterns and counts their top 12 bits (workgroup
// histograms in LDS, added into eight copies of a global histogram so the
// atomics spread); k_sel_gather finds the bin holding the median rank,
// counts that bin's patterns by their next 10 bits and gathers them into a
// list (one counter bump per workgroup); k_sel_list counts the listed
// patterns that share the median's 22-bit prefix by their low 10 bits; the
// row pass has already written the unscaled spectrum, and k_scale reads the
// exact pattern off that last histogram and scales X in place by
// 1 / sqrt(median / ln 2) (7-12 % faster than a second row pass that
// recomputed the rows from Y and wrote X scaled, the same bits).  Lengths the four-step form does not cover
// (powers of two below 2^6 or above 2^24 samples) take global Stockham
// passes and a three-round radix select over the spectrum.  Every counter
// and histogram is cleared by a kernel, so the call can be captured in a
// graph.
#include "internal.hpp"

#include <algorithm>

namespace fdas {

namespace {

constexpr int kPrepThreads = 256;

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// 4-point DFT in place: A_k = sum_n a_n exp(-2 pi i n k / 4)
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y), d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
    const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y), d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
    a0 = make_float2(s02.x + s13.x, s02.y + s13.y);
    a2 = make_float2(s02.x - s13.x, s02.y - s13.y);
    // -i d13 = (d13.y, -d13.x)
    a1 = make_float2(d02.x + d13.y, d02.y - d13.x);
    a3 = make_float2(d02.x - d13.y, d02.y + d13.x);
}

// 16-point DFT in registers, natural order in and out: n = 4 n1 + n2,
// k = k1 + 4 k2; inner 4-point DFTs over n1, factors exp(-2 pi i n2 k1 / 16),
// outer 4-point DFTs over n2.
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
    constexpr float c1 = 0.92387953251128674f;   // cos(pi / 8)
    constexpr float s1 = 0.38268343236508978f;   // sin(pi / 8)
    constexpr float h = 0.70710678118654752f;    // cos(pi / 4)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);   // v[4 k1 + n2]
    // exp(-2 pi i m / 16) for m = n2 k1 in {1, 2, 3, 4, 6, 9}
    const float2 w1 = make_float2(c1, -s1), w2 = make_float2(h, -h), w3 = make_float2(s1, -c1);
    const float2 w4 = make_float2(0.0f, -1.0f), w6 = make_float2(-h, -h), w9 = make_float2(-c1, s1);
    v[5] = cmulf(v[5], w1);   // k1 = 1, n2 = 1
    v[6] = cmulf(v[6], w2);   // k1 = 1, n2 = 2
    v[7] = cmulf(v[7], w3);   // k1 = 1, n2 = 3
    v[9] = cmulf(v[9], w2);   // k1 = 2, n2 = 1
    v[10] = cmulf(v[10], w4);
    v[11] = cmulf(v[11], w6);
    v[13] = cmulf(v[13], w3);   // k1 = 3, n2 = 1
    v[14] = cmulf(v[14], w6);
    v[15] = cmulf(v[15], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);   // v[4 k1 + k2]
    // natural order: X[k1 + 4 k2] = v[4 k1 + k2] (a 4 x 4 transpose)
    float2 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
}

__global__ void __launch_bounds__(kPrepThreads) k_stockham16(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                              int64_t N, int64_t Ns) {
    const int64_t j = blockIdx.x * (int64_t)kPrepThreads + threadIdx.x;
    const int64_t Q = N / 16;
    if (j >= Q) return;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = in[j + r * Q];
    const int64_t jm = j & (Ns - 1);
    if (Ns > 1) {
        // w = exp(-2 pi i jm / (16 Ns)); v[r] *= w^r, powers in double precision
        double s, c;
        sincospi(-2.0 * (double)jm / (double)(Ns * 16), &s, &c);
        double pr = c, pi = s;
#pragma unroll
        for (int r = 1; r < 16; ++r) {
            v[r] = cmulf(v[r], make_float2((float)pr, (float)pi));
            const double nr = pr * c - pi * s, ni = pr * s + pi * c;
            pr = nr;
            pi = ni;
        }
    }
    dft16(v);
    const int64_t base = (j / Ns) * Ns * 16 + jm;
#pragma unroll
    for (int r = 0; r < 16; ++r) out[base + r * Ns] = v[r];
}

template <int R>
__global__ void __launch_bounds__(kPrepThreads) k_stockham(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                            int64_t N, int64_t Ns) {
    const int64_t j = blockIdx.x * (int64_t)kPrepThreads + threadIdx.x;
    const int64_t Q = N / R;
    if (j >= Q) return;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[j + r * Q];
    const int64_t jm = j & (Ns - 1);
    if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            double s, c;
            sincospi(-2.0 * (double)(jm * r) / (double)(Ns * R), &s, &c);
            v[r] = cmulf(v[r], make_float2((float)c, (float)s));
        }
    }
    if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = make_float2(a.x + b.x, a.y + b.y);
        v[1] = make_float2(a.x - b.x, a.y - b.y);
    } else {
        const float2 a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
        const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y), d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
        const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y), d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
        v[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
        v[2] = make_float2(s02.x - s13.x, s02.y - s13.y);
        // -i d13 = (d13.y, -d13.x)
        v[1] = make_float2(d02.x + d13.y, d02.y - d13.x);
        v[3] = make_float2(d02.x - d13.y, d02.y + d13.x);
    }
    const int64_t base = (j / Ns) * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
}

// Real spectrum from the half-length complex transform; DC zeroed.
__global__ void __launch_bounds__(kPrepThreads) k_real_post(const float2 *__restrict__ Z, float2 *__restrict__ X,
                                                             int64_t N) {
    const int64_t k = blockIdx.x * (int64_t)kPrepThreads + threadIdx.x;
    if (k >= N) return;
    if (k == 0) {
        X[0] = make_float2(0.0f, 0.0f);
        return;
    }
    const float2 a = Z[k], b = Z[N - k];
    const float2 e = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));      // (Z[k] + conj Z[N-k]) / 2
    const float2 d = make_float2(0.5f * (a.x - b.x), 0.5f * (a.y + b.y));      // (Z[k] - conj Z[N-k]) / 2
    const float2 o = make_float2(d.y, -d.x);                                   // -i d
    double s, c;
    sincospi(-(double)k / (double)N, &s, &c);                                   // exp(-2 pi i k / (2N))
    const float2 t = cmulf(make_float2((float)c, (float)s), o);
    X[k] = make_float2(e.x + t.x, e.y + t.y);
}

// Radix-select state: [0] key prefix found so far, [1] rank left inside it.
struct SelState {
    uint32_t prefix;
    uint32_t rank;
};

__global__ void k_sel_init(SelState *st, uint32_t *hist, uint32_t rank) {
    for (int i = threadIdx.x; i < 2048; i += blockDim.x) hist[i] = 0;
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->rank = rank;
    }
}

__device__ __forceinline__ uint32_t power_bits(float2 v) { return __float_as_uint(v.x * v.x + v.y * v.y); }

// Pass p: keys whose bits above `shift + bits` equal the prefix, counted by
// bits [shift, shift + bits).
__global__ void __launch_bounds__(kPrepThreads) k_sel_hist(const float2 *__restrict__ X, int64_t N,
                                                            const SelState *st, uint32_t *hist, int shift,
                                                            int bits) {
    __shared__ uint32_t h[2048];
    const int nb = 1 << bits;
    for (int i = threadIdx.x; i < nb; i += kPrepThreads) h[i] = 0;
    __syncthreads();
    const uint32_t prefix = st->prefix;
    const int hi = shift + bits;   // bits above are fixed by the prefix
    for (int64_t k = 1 + blockIdx.x * (int64_t)kPrepThreads + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * kPrepThreads) {
        const uint32_t key = power_bits(X[k]);
        if (hi < 32 && (key >> hi) != prefix) continue;
        atomicAdd(&h[(key >> shift) & (nb - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kPrepThreads)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// One workgroup of 1024 threads, two bins each: an inclusive scan of the
// counts finds the bin holding the remaining rank (the one bin with
// exclusive sum <= rank < inclusive sum); the prefix is extended by it and
// the histogram cleared for the next pass.
__global__ void __launch_bounds__(1024) k_sel_pick(SelState *st, uint32_t *hist, int bits) {
    __shared__ uint32_t part[1024];
    const int nb = 1 << bits;
    const int t = threadIdx.x;
    const uint32_t c0 = 2 * t < nb ? hist[2 * t] : 0u, c1 = 2 * t + 1 < nb ? hist[2 * t + 1] : 0u;
    part[t] = c0 + c1;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
        const uint32_t v = t >= w ? part[t - w] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const uint32_t rank = st->rank;
    const uint32_t excl = part[t] - c0 - c1;   // counts of the bins before 2t
    __syncthreads();                             // every thread has read st->rank
    if (excl <= rank && rank < excl + c0) {
        st->prefix = (st->prefix << bits) | (uint32_t)(2 * t);
        st->rank = rank - excl;
    } else if (excl + c0 <= rank && rank < excl + c0 + c1) {
        st->prefix = (st->prefix << bits) | (uint32_t)(2 * t + 1);
        st->rank = rank - excl - c0;
    }
    for (int i = t; i < 2048; i += 1024) hist[i] = 0;
}

__global__ void __launch_bounds__(kPrepThreads) k_prep_scale(float2 *X, int64_t N, const SelState *st) {
    const int64_t k = blockIdx.x * (int64_t)kPrepThreads + threadIdx.x;
    if (k >= N) return;
    const double med = (double)__uint_as_float(st->prefix);
    const float s = (float)(1.0 / sqrt(med / 0.69314718055994530942));
    const float2 v = X[k];
    X[k] = make_float2(v.x * s, v.y * s);
}

// ---------------------------------------------------------------------------
// Four-step form: sub-transforms in LDS.
constexpr int kFsThreads = 1024;
constexpr int kFsPoints = 16384;          // complex values one workgroup transforms at once
constexpr int kFsMaxLen = 4096;
constexpr int kHistBins = 4096;           // top 12 bits of a power's bit pattern
constexpr int kHistShift = 20;
constexpr int kHistCopies = 8;            // copies of each global histogram (spread the atomics)
constexpr int kSubBins = 1024;            // next 10 bits, inside the median's top-12-bit bin
constexpr int kSelKeys = 16;              // keys per thread in the gather pass
// histogram words in the workspace: kHistCopies x (kHistBins + kSubBins)
// and the final low-bit histogram
constexpr int kHistWords = kHistCopies * (kHistBins + kSubBins) + kSubBins;

// 8-point DFT in registers, natural order: two radix-2 steps around 4-point DFTs
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
    constexpr float h = 0.70710678118654752f;
    float2 a[4] = {v[0], v[2], v[4], v[6]}, b[4] = {v[1], v[3], v[5], v[7]};
    dft4(a[0], a[1], a[2], a[3]);
    dft4(b[0], b[1], b[2], b[3]);
    // b[k] *= exp(-2 pi i k / 8)
    b[1] = cmulf(b[1], make_float2(h, -h));
    b[2] = make_float2(b[2].y, -b[2].x);
    b[3] = cmulf(b[3], make_float2(-h, -h));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = make_float2(a[k].x + b[k].x, a[k].y + b[k].y);
        v[k + 4] = make_float2(a[k].x - b[k].x, a[k].y - b[k].y);
    }
}

// 3-point DFT: A_k = sum_n a_n exp(-2 pi i n k / 3)
__device__ __forceinline__ void dft3(float2 &a0, float2 &a1, float2 &a2) {
    constexpr float r3 = 0.86602540378443865f;   // sqrt(3) / 2
    const float2 s = make_float2(a1.x + a2.x, a1.y + a2.y), d = make_float2(a1.x - a2.x, a1.y - a2.y);
    const float2 m = make_float2(a0.x - 0.5f * s.x, a0.y - 0.5f * s.y);
    a0 = make_float2(a0.x + s.x, a0.y + s.y);
    // -i r3 d = (r3 d.y, -r3 d.x)
    a1 = make_float2(m.x + r3 * d.y, m.y - r3 * d.x);
    a2 = make_float2(m.x - r3 * d.y, m.y + r3 * d.x);
}

template <int R>
__device__ __forceinline__ void dft_r(float2 (&v)[R]) {
    if constexpr (R == 16) dft16(v);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 3) dft3(v[0], v[1], v[2]);
    else {
        const float2 a = v[0], b = v[1];
        v[0] = make_float2(a.x + b.x, a.y + b.y);
        v[1] = make_float2(a.x - b.x, a.y - b.y);
    }
}

// LDS rows are padded by one element every 32 (pad(i) = i + i / 32): the
// first pass of a transform writes with a stride of R elements, which
// without padding would put 32 lanes of a wave on the same two banks.
__device__ __forceinline__ int pad32(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int row_words(int len) { return len + (len >> 5) + 1; }

// One radix-R Stockham pass over n_rows rows of length len in LDS (row r at
// buf + r * stride), sub-transform length Ns before the pass: butterfly j of
// a row reads j + q len / R, scales value q by exp(-2 pi i q (j mod Ns) /
// (Ns R)), and writes (j div Ns) Ns R + (j mod Ns) + q Ns.  Every input is
// read before the barrier and written after it, so one buffer serves.
template <int R>
__device__ __forceinline__ void lds_pass(float2 *buf, int stride, int len, int n_rows, int Ns) {
    constexpr int kMaxB = (kFsPoints + R * kFsThreads - 1) / (R * kFsThreads);
    const int nb = len / R, total = nb * n_rows;
    float2 v[kMaxB][R];
#pragma unroll
    for (int i = 0; i < kMaxB; ++i) {
        const int b = (int)threadIdx.x + i * kFsThreads;
        if (b < total) {
            const int row = b / nb, j = b - row * nb;
            const float2 *src = buf + row * stride;
#pragma unroll
            for (int q = 0; q < R; ++q) v[i][q] = src[pad32(j + q * nb)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxB; ++i) {
        const int b = (int)threadIdx.x + i * kFsThreads;
        if (b < total) {
            const int row = b / nb, j = b - row * nb;
            const int jm = j % Ns;
            if (Ns > 1) {
                float sn, cs;
                sincospif(-2.0f * (float)jm / (float)(Ns * R), &sn, &cs);
                const float2 w = make_float2(cs, sn);
                float2 wq = w;
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    v[i][q] = cmulf(v[i][q], wq);
                    if (q + 1 < R) wq = cmulf(wq, w);
                }
            }
            dft_r<R>(v[i]);
            float2 *dst = buf + row * stride;
            const int o = (j - jm) * R + jm;
#pragma unroll
            for (int q = 0; q < R; ++q) dst[pad32(o + q * Ns)] = v[i][q];
        }
    }
    __syncthreads();
}

// Forward FFT of n_rows rows of length len (2^a or 3 * 2^a, len <= 4096) in LDS.
__device__ __forceinline__ void lds_fft(float2 *buf, int stride, int len, int n_rows) {
    int Ns = 1;
    if (len % 3 == 0) {
        lds_pass<3>(buf, stride, len, n_rows, Ns);
        Ns = 3;
    }
    while (Ns * 16 <= len) {
        lds_pass<16>(buf, stride, len, n_rows, Ns);
        Ns *= 16;
    }
    if (Ns * 8 <= len) {
        lds_pass<8>(buf, stride, len, n_rows, Ns);
        Ns *= 8;
    }
    if (Ns * 4 <= len) {
        lds_pass<4>(buf, stride, len, n_rows, Ns);
        Ns *= 4;
    }
    if (Ns * 2 <= len) lds_pass<2>(buf, stride, len, n_rows, Ns);
}

struct FsState {
    uint32_t count;     // keys gathered by k_sel_compact
    uint32_t bin;       // the histogram bin holding the median
    uint32_t rank;      // the median's rank among the keys of that bin
    uint32_t key;       // the median's bit pattern
    float scale;        // 1 / sqrt(median / ln 2)
};

// Workgroups are dispatched to the 8 XCDs in turn (block b to XCD b mod 8),
// each XCD with its own L2.  Pass 1 reads C complex values (as little as 32
// bytes) of every row and pass 2 writes 32-byte runs of the spectrum, so
// neighbouring blocks share cache lines: the blocks of one XCD take
// consecutive indices, so that those lines meet in one L2 and leave it once.
__device__ __forceinline__ int xcd_local(int b, int nb) {
    const int full = nb & ~7;
    if (b >= full) return b;
    return (b & 7) * (full >> 3) + (b >> 3);
}

// Pass 1: the columns n2 in [c0, c0 + C) of z (viewed N1 x N2), FFT over n1,
// times e(-n2 k1 / N), to Y[k1][n2].  Workgroup 0 also clears the median
// state and histogram (used only by the later passes).
__global__ void __launch_bounds__(kFsThreads) k_cols(const float2 *__restrict__ z, float2 *__restrict__ Y, int N1,
                                                      int N2, int C, uint32_t *hist, FsState *state) {
    extern __shared__ float2 sh[];
    const int stride = row_words(N1);             // odd: the C rows start in different banks
    const int c0 = xcd_local((int)blockIdx.x, (int)gridDim.x) * C;
    const int64_t N = (int64_t)N1 * N2;
    // every workgroup clears its share of the histogram copies
    for (int i = blockIdx.x * kFsThreads + threadIdx.x; i < kHistWords; i += gridDim.x * kFsThreads) hist[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *state = FsState{0u, 0u, 0u, 0u, 0.0f};
    const int pts = C * N1;
    for (int i = threadIdx.x; i < pts; i += kFsThreads) {
        const int c = i % C, n1 = i / C;
        sh[c * stride + pad32(n1)] = z[(int64_t)N2 * n1 + c0 + c];
    }
    __syncthreads();
    lds_fft(sh, stride, N1, C);
    // times e(-n2 k1 / N): thread t meets k1 = k1_0 + q (1024 / C) of one
    // column (C divides 1024), so the factor starts at e(-n2 k1_0 / N) and
    // steps by e(-n2 (1024 / C) / N), both from exact integer ratios
    {
        const int c = threadIdx.x % C, k1_0 = threadIdx.x / C, dk = kFsThreads / C;
        const int n2 = c0 + c;
        float sn, cs;
        sincospif(-2.0f * (float)(((int64_t)n2 * k1_0) % N) / (float)N, &sn, &cs);
        float2 w = make_float2(cs, sn);
        sincospif(-2.0f * (float)(((int64_t)n2 * dk) % N) / (float)N, &sn, &cs);
        const float2 step = make_float2(cs, sn);
        for (int k1 = k1_0; k1 < N1; k1 += dk) {
            Y[(int64_t)k1 * N2 + n2] = cmulf(sh[c * stride + pad32(k1)], w);
            w = cmulf(w, step);
        }
    }
}

// Rows of workgroup g: slots 0..3 hold k1 = 4g + s, slots 4..7 their mirrors
// N1 - k1; in workgroup 0 slot 4 holds row N1 / 2 instead (row 0 is its own
// mirror).  N1 is a multiple of 8.
__device__ __forceinline__ int fs_row(int g, int s, int N1) {
    if (s < 4) return 4 * g + s;
    if (g == 0 && s == 4) return N1 / 2;
    return N1 - 4 * g - (s - 4);
}

// The real-spectrum bin of (slot s, k2) from the LDS rows (slot stride st).
__device__ __forceinline__ float2 fs_bin(const float2 *sh, int st, int g, int s, int k2, int N1, int N2) {
    const int k1 = fs_row(g, s, N1);
    int ps, pk;   // the slot and column of bin N - k
    if (k1 == 0) {
        ps = s;
        pk = k2 == 0 ? 0 : N2 - k2;
    } else if (g == 0 && s == 4) {
        ps = 4;
        pk = N2 - 1 - k2;
    } else {
        ps = s < 4 ? s + 4 : s - 4;
        pk = N2 - 1 - k2;
    }
    const int64_t k = (int64_t)k1 + (int64_t)N1 * k2;
    if (k == 0) return make_float2(0.0f, 0.0f);
    const float2 a = sh[s * st + pad32(k2)], b = sh[ps * st + pad32(pk)];
    const float2 e = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));   // (Z[k] + conj Z[N-k]) / 2
    const float2 d = make_float2(0.5f * (a.x - b.x), 0.5f * (a.y + b.y));   // (Z[k] - conj Z[N-k]) / 2
    const float2 o = make_float2(d.y, -d.x);                                // -i d
    const int64_t N = (int64_t)N1 * N2;
    float sn, cs;
    sincospif(-(float)k / (float)N, &sn, &cs);                              // exp(-2 pi i k / (2N))
    const float2 t = cmulf(make_float2(cs, sn), o);
    return make_float2(e.x + t.x, e.y + t.y);
}

// Inclusive scan of one value per thread over a 1024-thread workgroup
// (wave prefix sums by shuffles, then the 16 wave totals).
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        uint32_t t = lane < kFsThreads / 64 ? wsum[lane] : 0u;
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            const uint32_t u = __shfl_up(t, d);
            if (lane >= d) t += u;
        }
        if (lane < kFsThreads / 64) wsum[lane] = t;
    }
    __syncthreads();
    const uint32_t r = v + (w > 0 ? wsum[w - 1] : 0u);
    __syncthreads();
    return r;
}

// Gather pass: every workgroup finds the top-12-bit bin holding the median
// rank (from the histogram copies), then, over its kSelKeys x 1024 keys,
// (a) counts the keys of that bin by their next 10 bits into the copies of
// the sub-histogram and (b) appends them to `list` (one counter bump per
// workgroup).
__global__ void __launch_bounds__(kFsThreads) k_sel_gather(const uint32_t *__restrict__ keys, int64_t n,
                                                            uint32_t *__restrict__ hist, uint32_t rank,
                                                            uint32_t *__restrict__ list, FsState *state) {
    __shared__ uint32_t wsum[kFsThreads / 64];
    __shared__ uint32_t sub[kSubBins];
    __shared__ uint32_t s_bin, s_base;
    const int t = threadIdx.x;
    // 1. the median's bin: four bins per thread, summed over the copies
    uint32_t c[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < kHistCopies; ++k) v += hist[k * kHistBins + 4 * t + q];
        c[q] = v;
        sum += v;
    }
    sub[t] = 0;
    uint32_t excl = block_scan(sum, wsum) - sum;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (excl <= rank && rank < excl + c[q]) {
            s_bin = 4 * t + q;
            if (blockIdx.x == 0) {
                state->bin = 4 * t + q;
                state->rank = rank - excl;
            }
        }
        excl += c[q];
    }
    __syncthreads();
    const uint32_t bin = s_bin;
    // 2. this workgroup's keys (consecutive threads, consecutive keys)
    const int64_t base = (int64_t)blockIdx.x * kSelKeys * kFsThreads;
    uint32_t mine[kSelKeys];
    uint32_t hits = 0;
#pragma unroll
    for (int q = 0; q < kSelKeys; ++q) {
        const int64_t i = base + (int64_t)q * kFsThreads + t;
        mine[q] = i < n ? keys[i] : 0xffffffffu;
        if (i < n && (mine[q] >> kHistShift) == bin) ++hits;
    }
#pragma unroll
    for (int q = 0; q < kSelKeys; ++q)
        if ((mine[q] >> kHistShift) == bin && base + (int64_t)q * kFsThreads + t < n)
            atomicAdd(&sub[(mine[q] >> 10) & (kSubBins - 1)], 1u);
    const uint32_t incl = block_scan(hits, wsum);
    if (t == kFsThreads - 1) s_base = incl ? atomicAdd(&state->count, incl) : 0u;
    __syncthreads();
    uint32_t pos = s_base + incl - hits;
#pragma unroll
    for (int q = 0; q < kSelKeys; ++q)
        if ((mine[q] >> kHistShift) == bin && base + (int64_t)q * kFsThreads + t < n) list[pos++] = mine[q];
    uint32_t *sc = hist + kHistCopies * kHistBins + (blockIdx.x % kHistCopies) * kSubBins;
    if (sub[t]) atomicAdd(&sc[t], sub[t]);
}

// The 22-bit prefix of the median (its top-12-bit bin and the sub-bin that
// holds the remaining rank, from the sub-histogram copies) and the rank left
// inside it; every workgroup of the list pass computes it.
__device__ __forceinline__ void sub_prefix(const uint32_t *hist, const FsState *state, uint32_t *wsum,
                                           uint32_t *s_prefix, uint32_t *s_rank) {
    const int t = threadIdx.x;
    const uint32_t bin = state->bin, rank0 = state->rank;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kHistCopies; ++k) c += hist[kHistCopies * kHistBins + k * kSubBins + t];
    const uint32_t excl = block_scan(c, wsum) - c;
    if (excl <= rank0 && rank0 < excl + c) {
        *s_prefix = (bin << 10) | (uint32_t)t;
        *s_rank = rank0 - excl;
    }
    __syncthreads();
}

// List pass: the gathered keys with the median's 22-bit prefix, counted by
// their low 10 bits into the final histogram (few keys: no copies needed).
__global__ void __launch_bounds__(kFsThreads) k_sel_list(const uint32_t *__restrict__ list,
                                                          uint32_t *__restrict__ hist, FsState *state) {
    __shared__ uint32_t wsum[kFsThreads / 64];
    __shared__ uint32_t h[kSubBins];
    __shared__ uint32_t s_prefix, s_rank;
    const int t = threadIdx.x;
    h[t] = 0;
    sub_prefix(hist, state, wsum, &s_prefix, &s_rank);
    const uint32_t prefix = s_prefix, n = state->count;
    for (uint32_t i = blockIdx.x * kFsThreads + t; i < n; i += gridDim.x * kFsThreads) {
        const uint32_t key = list[i];
        if ((key >> 10) == prefix) atomicAdd(&h[key & (kSubBins - 1)], 1u);
    }
    __syncthreads();
    uint32_t *fin = hist + kHistCopies * (kHistBins + kSubBins);
    if (h[t]) atomicAdd(&fin[t], h[t]);
}

// The median's bit pattern from the final histogram (each workgroup of the
// last row pass) and the scale 1 / sqrt(median / ln 2).
__device__ __forceinline__ float median_scale(const uint32_t *hist, const FsState *state, uint32_t *wsum,
                                              uint32_t *s_prefix, uint32_t *s_rank, float *s_scale) {
    const int t = threadIdx.x;
    sub_prefix(hist, state, wsum, s_prefix, s_rank);
    const uint32_t *fin = hist + kHistCopies * (kHistBins + kSubBins);
    const uint32_t c = fin[t], rank = *s_rank;
    const uint32_t excl = block_scan(c, wsum) - c;
    if (excl <= rank && rank < excl + c) {
        const uint32_t key = (*s_prefix << 10) | (uint32_t)t;
        const double med = (double)__uint_as_float(key);
        *s_scale = (float)(1.0 / sqrt(med / 0.69314718055994530942));
    }
    __syncthreads();
    return *s_scale;
}

// Pass 2: the eight rows of workgroup g from Y, FFT over n2; the power bit
// patterns to keys[k1 * N2 + k2] (DC: all ones, above every power) with
// their top-bit histogram, and the unscaled spectrum X[k] in natural order.
__global__ void __launch_bounds__(kFsThreads) k_rows(const float2 *__restrict__ Y, int N1, int N2,
                                                      uint32_t *__restrict__ keys, uint32_t *__restrict__ hist,
                                                      float2 *__restrict__ X) {
    extern __shared__ float2 sh[];
    const int st = row_words(N2);
    const int g = xcd_local((int)blockIdx.x, (int)gridDim.x);
    uint32_t *lh = reinterpret_cast<uint32_t *>(sh + 8 * st);
    for (int i = threadIdx.x; i < kHistBins; i += kFsThreads) lh[i] = 0;
    for (int i = threadIdx.x; i < 8 * N2; i += kFsThreads) {
        const int s = i / N2, n2 = i - s * N2;
        sh[s * st + pad32(n2)] = Y[(int64_t)fs_row(g, s, N1) * N2 + n2];
    }
    __syncthreads();
    lds_fft(sh, st, N2, 8);
    for (int i = threadIdx.x; i < 8 * N2; i += kFsThreads) {
        const int s = i / N2, k2 = i - s * N2;
        const int k1 = fs_row(g, s, N1);
        const float2 x = fs_bin(sh, st, g, s, k2, N1, N2);
        const bool dc = k1 == 0 && k2 == 0;
        const uint32_t key = dc ? 0xffffffffu : __float_as_uint(x.x * x.x + x.y * x.y);
        keys[(int64_t)k1 * N2 + k2] = key;
        atomicAdd(&lh[key >> kHistShift], 1u);
    }
    // consecutive threads take consecutive k1 (four rows ascending, then
    // their mirrors, also ascending in k1) for one k2
    for (int i = threadIdx.x; i < 8 * N2; i += kFsThreads) {
        const int half = i / (4 * N2), r = i - half * 4 * N2;
        const int q = r & 3, k2 = r >> 2;
        const int s = half == 0 ? q : 4 + (3 - q);
        if (g == 0 && s == 4) continue;            // row N1 / 2: written below
        X[(int64_t)fs_row(g, s, N1) + (int64_t)N1 * k2] = fs_bin(sh, st, g, s, k2, N1, N2);
    }
    if (g == 0) {
        for (int k2 = threadIdx.x; k2 < N2; k2 += kFsThreads)
            X[(int64_t)(N1 / 2) + (int64_t)N1 * k2] = fs_bin(sh, st, 0, 4, k2, N1, N2);
    }
    __syncthreads();
    uint32_t *hc = hist + (g % kHistCopies) * kHistBins;
    for (int i = threadIdx.x; i < kHistBins; i += kFsThreads)
        if (lh[i]) atomicAdd(&hc[i], lh[i]);
}

// Pass 3: X scaled in place by the median's factor (each workgroup reads the
// median from the final histogram).
__global__ void __launch_bounds__(kFsThreads) k_scale(float2 *__restrict__ X, int64_t N,
                                                       const uint32_t *__restrict__ hist, const FsState *state) {
    __shared__ uint32_t wsum[kFsThreads / 64];
    __shared__ uint32_t s_prefix, s_rank;
    __shared__ float s_scale;
    const float sc = median_scale(hist, state, wsum, &s_prefix, &s_rank, &s_scale);
    for (int64_t i = blockIdx.x * (int64_t)kFsThreads + threadIdx.x; i < N; i += (int64_t)gridDim.x * kFsThreads) {
        const float2 x = X[i];
        X[i] = make_float2(x.x * sc, x.y * sc);
    }
}

// The four-step factorisation of N: N = 2^a -> N2 = 2^floor(a/2),
// N1 = 2^ceil(a/2); N = 3 * 2^a -> N2 = 2^ceil(a/2), N1 = 3 * 2^floor(a/2)
// (N1 > N2); N1 <= 4096 and a multiple of 8, 2 <= N2 <= 2048 (eight rows of
// N2 fill a workgroup's LDS), or false.
bool fs_split(int64_t N, int *n1, int *n2) {
    const bool three = N % 3 == 0;
    const int64_t p = three ? N / 3 : N;
    if (p <= 0 || (p & (p - 1)) != 0) return false;
    int a = 0;
    while (((int64_t)1 << a) < p) ++a;
    const int64_t N2 = three ? (int64_t)1 << ((a + 1) / 2) : (int64_t)1 << (a / 2);
    const int64_t N1 = N / N2;
    if (N1 > kFsMaxLen || N1 % 8 != 0 || N2 < 2 || N2 > 2048) return false;
    *n1 = (int)N1;
    *n2 = (int)N2;
    return true;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kPrepThreads - 1) / kPrepThreads); }

}  // namespace

size_t prep_workspace_bytes(int64_t n_t) {
    const int64_t N = n_t / 2;
    // four-step: Y (N complex), keys and gathered keys (N each); global
    // passes: two N-complex buffers; both followed by histogram and state
    return (size_t)2 * N * sizeof(float2) + kHistWords * sizeof(uint32_t) + 256;
}

bool prep_length_supported(int64_t n_t) {
    if (n_t < 4 || n_t % 4 != 0 || n_t > ((int64_t)1 << 28)) return false;
    int n1, n2;
    if (fs_split(n_t / 2, &n1, &n2)) return true;
    return (n_t & (n_t - 1)) == 0;   // global passes: powers of two
}

namespace {
hipError_t launch_fourstep(const float *series, int64_t N, int N1, int N2, float2 *X, void *ws, hipStream_t st) {
    auto *Y = static_cast<float2 *>(ws);
    auto *keys = reinterpret_cast<uint32_t *>(Y + N);
    uint32_t *list = keys + N;
    uint32_t *hist = list + N;
    auto *state = reinterpret_cast<FsState *>(hist + kHistWords);
    int C = 1;
    while (2 * C * N1 <= kFsPoints && 2 * C <= N2 && 2 * C <= kFsThreads) C *= 2;
    const size_t lds_cols = (size_t)C * row_words(N1) * sizeof(float2);
    const size_t lds_rows = (size_t)8 * row_words(N2) * sizeof(float2) + kHistBins * sizeof(uint32_t);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cols),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_cols);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_rows);
    if (e != hipSuccess) return e;
    const auto *z = reinterpret_cast<const float2 *>(series);
    hipLaunchKernelGGL(k_cols, dim3((unsigned)(N2 / C)), dim3(kFsThreads), lds_cols, st, z, Y, N1, N2, C, hist,
                       state);
    hipLaunchKernelGGL(k_rows, dim3((unsigned)(N1 / 8)), dim3(kFsThreads), lds_rows, st, Y, N1, N2, keys, hist,
                       X);
    // the median of the N - 1 powers k >= 1: rank (N - 2) / 2 from below (the
    // DC key sits above every power)
    const int64_t per = (int64_t)kSelKeys * kFsThreads;
    hipLaunchKernelGGL(k_sel_gather, dim3((unsigned)((N + per - 1) / per)), dim3(kFsThreads), 0, st, keys, N, hist,
                       (uint32_t)((N - 2) / 2), list, state);
    hipLaunchKernelGGL(k_sel_list, dim3(256), dim3(kFsThreads), 0, st, list, hist, state);
    hipLaunchKernelGGL(k_scale, dim3((unsigned)std::min<int64_t>(N / kFsThreads + 1, 1024)), dim3(kFsThreads), 0, st,
                       X, N, hist, state);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_prepare(const float *series, int64_t n_t, void *out, void *ws, hipStream_t st) {
    const int64_t N = n_t / 2;
    int N1, N2;
    if (fs_split(N, &N1, &N2)) return launch_fourstep(series, N, N1, N2, static_cast<float2 *>(out), ws, st);
    auto *bufA = static_cast<float2 *>(ws);
    float2 *bufB = bufA + N;
    auto *hist = reinterpret_cast<uint32_t *>(bufB + N);
    auto *state = reinterpret_cast<SelState *>(hist + 2048);
    auto *X = static_cast<float2 *>(out);
    // complex FFT of length N: radix-16 passes, then radix 4, then radix 2
    const float2 *src = reinterpret_cast<const float2 *>(series);
    float2 *dst = bufA;
    int64_t Ns = 1;
    while (Ns * 16 <= N) {
        hipLaunchKernelGGL(k_stockham16, dim3(blocks_for(N / 16)), dim3(kPrepThreads), 0, st, src, dst, N, Ns);
        Ns *= 16;
        src = dst;
        dst = (dst == bufA) ? bufB : bufA;
    }
    while (Ns * 4 <= N) {
        hipLaunchKernelGGL(k_stockham<4>, dim3(blocks_for(N / 4)), dim3(kPrepThreads), 0, st, src, dst, N, Ns);
        Ns *= 4;
        src = dst;
        dst = (dst == bufA) ? bufB : bufA;
    }
    if (Ns < N) {
        hipLaunchKernelGGL(k_stockham<2>, dim3(blocks_for(N / 2)), dim3(kPrepThreads), 0, st, src, dst, N, Ns);
        src = dst;
    }
    hipLaunchKernelGGL(k_real_post, dim3(blocks_for(N)), dim3(kPrepThreads), 0, st, src, X, N);
    // median of the N - 1 powers k >= 1 (rank (N - 2) / 2, N - 1 odd)
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, st, state, hist, (uint32_t)((N - 2) / 2));
    const unsigned hb = std::min<unsigned>(blocks_for(N), 2048);
    const int shifts[3] = {21, 10, 0}, widths[3] = {11, 11, 10};
    for (int p = 0; p < 3; ++p) {
        hipLaunchKernelGGL(k_sel_hist, dim3(hb), dim3(kPrepThreads), 0, st, X, N, state, hist, shifts[p],
                           widths[p]);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, st, state, hist, widths[p]);
    }
    hipLaunchKernelGGL(k_prep_scale, dim3(blocks_for(N)), dim3(kPrepThreads), 0, st, X, N, state);
    return hipGetLastError();
}

}  // namespace fdas
