// FP8 (OCP e4m3) storage form of the vector-ALU transforms.
//
// e4m3 holds 3 mantissa bits and values up to 448, so every stored stage
// carries a power-of-two scale: before a stage is written to LDS (or kept in
// registers) the workgroup takes the largest |re| / |im| of that stage and
// stores fp8(v 2^e) with 2^e the largest power of two keeping it <= 448;
// loading multiplies by 2^-e.  Scaling by powers of two is exact, so the only
// error is the e4m3 rounding itself (round to nearest even, relative error at
// most 2^-4 of the value for normal numbers).  Arithmetic stays FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "fft_valu.hpp"

namespace fdas {

// e4m3 pair: re in the low byte, im in the high byte.
struct fp8c {
    uint16_t bits;
};

__device__ __forceinline__ uint16_t fp8_pack(float re, float im) {
    return (uint16_t)(__builtin_amdgcn_cvt_pk_fp8_f32(re, im, 0, false) & 0xFFFF);
}
__device__ __forceinline__ cpx<float> fp8_unpack(uint16_t b) {
    return {__builtin_amdgcn_cvt_f32_fp8((int)b, 0), __builtin_amdgcn_cvt_f32_fp8((int)b, 1)};
}

// 2^e for the largest e with amax 2^e <= 448; 1 for amax = 0 and for a
// non-finite amax (NaN / Inf then propagate as the e4m3 NaN).
__device__ __forceinline__ float fp8_scale_for(float amax) {
    if (!(amax > 0.0f) || !(amax <= FLT_MAX)) return 1.0f;
    int e = (int)floorf(log2f(448.0f / amax));
    // log2f may be off by one ulp at exact powers: correct both ways
    while (ldexpf(amax, e) > 448.0f) --e;
    while (ldexpf(amax, e + 1) <= 448.0f) ++e;
    e = e > 126 ? 126 : (e < -126 ? -126 : e);
    return ldexpf(1.0f, e);
}

// Workgroup-wide max of a non-negative per-thread value.  slot alternates
// between two LDS words so that no barrier is needed to clear it: the word
// for the next call is cleared here, two barriers before it is used.
__device__ __forceinline__ float block_amax(float v, unsigned int *slots, int &slot) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&slots[slot], __float_as_uint(v));   // v >= 0 or NaN
    __syncthreads();
    const float r = __uint_as_float(slots[slot]);
    if (threadIdx.x == 0) slots[slot ^ 1] = 0u;
    slot ^= 1;
    return r;
}

__device__ __forceinline__ float cmax_abs(cpx<float> v) { return fmaxf(fabsf(v.re), fabsf(v.im)); }

// One Stockham pass with the stage written as scaled e4m3 (same index
// scheme as stockham_pass): outputs are formed in registers, the workgroup
// amax fixes the scale, then the stage goes through LDS.
template <int R, int S, int LOG2L, int Ls, bool LAST>
__device__ __forceinline__ void stockham_pass_fp8(cpx<float> (&a)[16], fp8c *lds, const cpx<float> *tw, int t,
                                                  unsigned int *slots, int &slot) {
    constexpr int L = 1 << LOG2L;
    constexpr int TH = L / 16;
    constexpr int G = 16 / R;
    constexpr int STEP = L / (Ls * R);
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int v = t + i * TH;
        cpx<float> b[R];
#pragma unroll
        for (int k = 0; k < R; ++k) b[k] = a[i + k * G];
        const int jj = v & (Ls - 1);
        if constexpr (Ls > 1) {
            const int e1 = jj * STEP;
#pragma unroll
            for (int k = 1; k < R; ++k) {
                const cpx<float> w = tw[e1 * k];
                b[k] = S < 0 ? cmul(b[k], w) : cmulc(b[k], w);
            }
        }
        dft<R, S>(b);
#pragma unroll
        for (int k = 0; k < R; ++k) a[i + k * G] = b[k];
    }
    if constexpr (!LAST) {
        float m = 0.0f;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) m = fmaxf(m, cmax_abs(a[kk]));
        const float sc = fp8_scale_for(block_amax(m, slots, slot));
        const float inv = 1.0f / sc;   // exact: a power of two
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int v = t + i * TH;
            const int jj = v & (Ls - 1);
            const int o = (v - jj) * R + jj;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const cpx<float> x = a[i + k * G];
                lds[lds_pad(o + k * Ls)] = fp8c{fp8_pack(x.re * sc, x.im * sc)};
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const cpx<float> x = fp8_unpack(lds[lds_pad(t + kk * TH)].bits);
            a[kk] = {x.re * inv, x.im * inv};
        }
        __syncthreads();
    }
}

template <int S, int LOG2L, int P>
__device__ __forceinline__ void run_passes_fp8(cpx<float> (&a)[16], fp8c *lds, const cpx<float> *tw, int t,
                                               unsigned int *slots, int &slot) {
    using sch = schedule<LOG2L>;
    if constexpr (P < sch::npass) {
        stockham_pass_fp8<sch::radix(P), S, LOG2L, sch::sublen(P), P == sch::npass - 1>(a, lds, tw, t, slots, slot);
        run_passes_fp8<S, LOG2L, P + 1>(a, lds, tw, t, slots, slot);
    }
}

template <int S, int LOG2L>
__device__ __forceinline__ void fft_fp8(cpx<float> (&a)[16], fp8c *lds, const cpx<float> *tw, int t,
                                        unsigned int *slots, int &slot) {
    run_passes_fp8<S, LOG2L, 0>(a, lds, tw, t, slots, slot);
}

}  // namespace fdas
