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
// z[m] = x[2m] + i x[2m+1] (the series reinterpreted, no copy); a complex FFT
// of length N in Stockham autosort passes over global memory (radix 16 while
// it fits, then radix 4, then one radix-2 pass if needed; thread j of a pass
// with sub-transform length Ns reads R values j + r N / R, twiddles them by
// exp(-2 pi i (j mod Ns) r / (Ns R)), takes an R-point DFT and writes them to
// (j div Ns) Ns R + (j mod Ns) + r Ns, so the output is in natural order
// after the last pass).  The 16-point DFT runs in registers as 4 x 4 with
// the internal factors exp(-2 pi i m / 16) as constants; the pass twiddles
// come from one double-precision sincospi per thread and its powers formed
// in double precision.  The real
// spectrum follows from E[k] = (Z[k] + conj Z[N-k]) / 2 (even samples),
// O[k] = -i (Z[k] - conj Z[N-k]) / 2 (odd samples), X[k] = E[k] + e(-k / 2N) O[k].
//
// Median.  Exact selection of the middle power among the N - 1 bins k >= 1
// (an odd count for N a power of two) by a radix select on the powers' bit
// patterns (non-negative floats order like their patterns): three histogram
// passes over 11, 11 and 10 bits, each followed by one workgroup that finds
// the bin holding the remaining rank.  Histograms and state are cleared by
// kernels, so the call can be captured in a graph.
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

unsigned blocks_for(int64_t n) { return (unsigned)((n + kPrepThreads - 1) / kPrepThreads); }

}  // namespace

size_t prep_workspace_bytes(int64_t n_t) {
    const int64_t N = n_t / 2;
    return (size_t)2 * N * sizeof(float2) + 2048 * sizeof(uint32_t) + 256;
}

hipError_t launch_prepare(const float *series, int64_t n_t, void *out, void *ws, hipStream_t st) {
    const int64_t N = n_t / 2;
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
