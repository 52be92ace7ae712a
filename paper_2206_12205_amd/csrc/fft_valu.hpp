// Vector-ALU FFT building blocks for one workgroup-wide transform.
//
// A transform of length L = 2^LOG2L is held by T = L / 16 threads, 16 complex
// points each: thread t holds x[t + kk * T], kk in [0, 16).  Passes follow
// the Stockham autosort scheme (natural order in and out, no bit reversal):
// a radix-R pass with sub-length Ls lets virtual thread v in [0, L/R) read
// x[v + k L/R], twiddle by W_{Ls R}^{(v mod Ls) k}, apply a radix-R DFT and
// write y[(v - v mod Ls) R + v mod Ls + k Ls].  With 16 points per thread the
// read set of every pass, and the write set of the last pass, is exactly the
// thread's own {t + kk T}: the first pass reads registers and the last pass
// writes registers; the passes in between exchange through LDS.
//
// Radix schedule: 16-point passes, plus one 2/4/8-point pass for the
// remaining bits (placed last, where it needs the fewest twiddles).
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

template <class R>
struct cpx {
    R re, im;
};

template <class R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <class R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// cos / sin of 2 pi e / 16, e in [0, 16)
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// v * exp(S 2 pi i e / 16); e is a constant after unrolling, so the branches fold.
template <int S, class R>
__device__ __forceinline__ cpx<R> rot16(cpx<R> v, int e) {
    e &= 15;
    if (e == 0) return v;
    if (e == 8) return {-v.re, -v.im};
    if (e == 4) return S > 0 ? cpx<R>{-v.im, v.re} : cpx<R>{v.im, -v.re};
    if (e == 12) return S > 0 ? cpx<R>{v.im, -v.re} : cpx<R>{-v.im, v.re};
    const R c = (R)kCos16[e];
    const R s = (R)(S * kSin16[e]);
    return {v.re * c - v.im * s, v.re * s + v.im * c};
}

template <int S, class R>
__device__ __forceinline__ void dft2(cpx<R> *a) {
    cpx<R> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

template <int S, class R>
__device__ __forceinline__ void dft4(cpx<R> *a) {
    const cpx<R> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const cpx<R> t2 = cadd(a[1], a[3]), t3 = csub(a[1], a[3]);
    // X1 = t1 + (S i) t3, X3 = t1 - (S i) t3
    const cpx<R> it3 = S > 0 ? cpx<R>{-t3.im, t3.re} : cpx<R>{t3.im, -t3.re};
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, it3);
    a[3] = csub(t1, it3);
}

// Composite DFT of length R1 * R2 in registers: n = R2 n1 + n2, k = k1 + R1 k2,
// X[k] = sum_n2 W_R2^{n2 k2} W_R^{n2 k1} sum_n1 W_R1^{n1 k1} x[R2 n1 + n2].
template <int R, int S, class T>
__device__ __forceinline__ void dft(cpx<T> *a);

template <int R1, int R2, int S, class T>
__device__ __forceinline__ void dft_comp(cpx<T> *a) {
    constexpr int N = R1 * R2;
    cpx<T> b[N];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        cpx<T> u[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) u[n1] = a[R2 * n1 + n2];
        dft<R1, S>(u);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) b[k1 * R2 + n2] = rot16<S>(u[k1], (n2 * k1 * (16 / N)));
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        dft<R2, S>(&b[k1 * R2]);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = b[k1 * R2 + k2];
    }
}

template <int R, int S, class T>
__device__ __forceinline__ void dft(cpx<T> *a) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        dft2<S>(a);
    } else if constexpr (R == 4) {
        dft4<S>(a);
    } else if constexpr (R == 8) {
        dft_comp<2, 4, S>(a);
    } else if constexpr (R == 16) {
        dft_comp<4, 4, S>(a);
    }
}

// LDS index padding: one spare slot per 16 keeps strided writes conflict-light.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

// Storage conversions between the compute type and the LDS / register
// storage type of the precision form.
template <class R, class Sto>
struct store_cvt;

template <class R>
struct store_cvt<R, cpx<R>> {
    static __device__ __forceinline__ cpx<R> put(cpx<R> v) { return v; }
    static __device__ __forceinline__ cpx<R> get(cpx<R> v) { return v; }
};

// bfloat16 pair packed in 32 bits: re in the low half, im in the high half.
struct bf16c {
    uint32_t bits;
};
__device__ __forceinline__ float bf16_lo(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t b) { return __uint_as_float(b & 0xffff0000u); }
__device__ __forceinline__ uint32_t bf16_pack(float re, float im) {
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    bf2 v;
    v.x = (__bf16)re;   // round to nearest even (v_cvt_pk_bf16_f32)
    v.y = (__bf16)im;
    return __builtin_bit_cast(uint32_t, v);
}

template <>
struct store_cvt<float, bf16c> {
    static __device__ __forceinline__ bf16c put(cpx<float> v) { return {bf16_pack(v.re, v.im)}; }
    static __device__ __forceinline__ cpx<float> get(bf16c v) {
        return {bf16_lo(v.bits), bf16_hi(v.bits)};
    }
};

// One Stockham pass.  Template arguments fix the radix, sign, length, the
// sub-length Ls and whether this is the last pass.
template <int R, int S, int LOG2L, int Ls, bool LAST, class T, class Sto>
__device__ __forceinline__ void stockham_pass(cpx<T> (&a)[16], Sto *lds, const cpx<T> *tw, int t) {
    constexpr int L = 1 << LOG2L;
    constexpr int TH = L / 16;
    constexpr int G = 16 / R;          // virtual threads per thread
    constexpr int STEP = L / (Ls * R);  // twiddle table stride
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int v = t + i * TH;
        cpx<T> b[R];
#pragma unroll
        for (int k = 0; k < R; ++k) b[k] = a[i + k * G];
        const int jj = v & (Ls - 1);
        if constexpr (Ls > 1) {
            const int e1 = jj * STEP;
#pragma unroll
            for (int k = 1; k < R; ++k) {
                const cpx<T> w = tw[e1 * k];
                b[k] = S < 0 ? cmul(b[k], w) : cmulc(b[k], w);
            }
        }
        dft<R, S>(b);
        if constexpr (LAST) {
#pragma unroll
            for (int k = 0; k < R; ++k) a[i + k * G] = b[k];
        } else {
            const int o = (v - jj) * R + jj;
#pragma unroll
            for (int k = 0; k < R; ++k) lds[lds_pad(o + k * Ls)] = store_cvt<T, Sto>::put(b[k]);
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) a[kk] = store_cvt<T, Sto>::get(lds[lds_pad(t + kk * TH)]);
        __syncthreads();
    }
}

template <int LOG2L>
struct schedule {
    static constexpr int n16 = LOG2L / 4;
    static constexpr int rem = LOG2L % 4;
    static constexpr int npass = n16 + (rem ? 1 : 0);
    static constexpr int radix(int p) { return p < n16 ? 16 : (1 << rem); }
    static constexpr int sublen(int p) { return p == 0 ? 1 : sublen(p - 1) * radix(p - 1); }
};

template <int S, int LOG2L, int P, class T, class Sto>
__device__ __forceinline__ void run_passes(cpx<T> (&a)[16], Sto *lds, const cpx<T> *tw, int t) {
    using sch = schedule<LOG2L>;
    if constexpr (P < sch::npass) {
        stockham_pass<sch::radix(P), S, LOG2L, sch::sublen(P), P == sch::npass - 1>(a, lds, tw, t);
        run_passes<S, LOG2L, P + 1>(a, lds, tw, t);
    }
}

// Whole transform of the workgroup's L points held 16 per thread.
// S = -1: forward, exp(-2 pi i n k / L); S = +1: inverse without the 1/L.
template <int S, int LOG2L, class T, class Sto>
__device__ __forceinline__ void fft(cpx<T> (&a)[16], Sto *lds, const cpx<T> *tw, int t) {
    run_passes<S, LOG2L, 0>(a, lds, tw, t);
}

}  // namespace fdas
