// Overlap-save correlation of a spectrum with the template bank: the f-fdot
// plane (Section "Detailed explanation": split the long spectrum into
// windows, transform each, multiply by every template's transform, inverse
// transform, keep the central region and discard the contaminated edges).
//
// One workgroup owns one segment s and a chunk of consecutive templates:
//   1. load the window X[s V - M/2 .. s V - M/2 + L) (zeros outside [0, N)),
//      16 points per thread, coalesced;
//   2. forward FFT (Stockham passes, LDS between passes); the spectrum of
//      the segment stays in registers in the storage precision;
//   3. for each template j of the chunk: multiply by H_j (read from the bank,
//      which already holds the 1/L of the inverse transform), inverse FFT,
//      |.|^2, and store the V central outputs p in [M/2, L - M/2) to
//      plane[j, s V + p - M/2] with non-temporal coalesced stores.
// Workgroup b takes template chunk b mod n_chunks and segment b / n_chunks,
// so consecutive workgroups (which the dispatcher spreads over the XCDs)
// share a segment, and with n_chunks a multiple of the XCD count each XCD's
// L2 serves a fixed subset of the bank.
#include "fft_valu.hpp"
#include "internal.hpp"
#include "plane_io.hpp"

namespace fdas {

// Bank element -> compute complex.
template <class T, class B>
__device__ __forceinline__ cpx<T> bank_get(const B *bank, int64_t i);
template <>
__device__ __forceinline__ cpx<float> bank_get<float, cpx<float>>(const cpx<float> *b, int64_t i) {
    return b[i];
}
template <>
__device__ __forceinline__ cpx<double> bank_get<double, cpx<double>>(const cpx<double> *b, int64_t i) {
    return b[i];
}
template <>
__device__ __forceinline__ cpx<float> bank_get<float, bf16c>(const bf16c *b, int64_t i) {
    const uint32_t v = b[i].bits;
    return {bf16_lo(v), bf16_hi(v)};
}

template <int LOG2L, class T, class Sto, class PT>
__global__ void __launch_bounds__((1 << LOG2L) / 16)
correlate_valu(const float *__restrict__ spec, int64_t n, const Sto *__restrict__ bank,
               const cpx<T> *__restrict__ tw, PT *__restrict__ plane, int32_t M, int32_t V,
               int32_t n_z, int32_t z_chunk, int32_t n_chunks) {
    constexpr int L = 1 << LOG2L;
    constexpr int TH = L / 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Sto *lds = reinterpret_cast<Sto *>(smem_raw);

    const int t = threadIdx.x;
    const int chunk = blockIdx.x % n_chunks;
    const int64_t s = blockIdx.x / n_chunks;
    const int j0 = chunk * z_chunk;
    const int j1 = min(j0 + z_chunk, n_z);
    if (j0 >= j1) return;
    const int64_t base = s * (int64_t)V - M / 2;

    cpx<T> a[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        const int64_t idx = base + t + kk * TH;
        if (idx >= 0 && idx < n) {
            const float2 v = reinterpret_cast<const float2 *>(spec)[idx];
            a[kk] = {(T)v.x, (T)v.y};
        } else {
            a[kk] = {(T)0, (T)0};
        }
    }
    fft<-1, LOG2L>(a, lds, tw, t);

    Sto shat[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) shat[kk] = store_cvt<T, Sto>::put(a[kk]);

    const int half = M / 2;
    for (int j = j0; j < j1; ++j) {
        const Sto *hb = bank + (int64_t)j * L;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const cpx<T> h = bank_get<T, Sto>(hb, t + kk * TH);
            a[kk] = cmul(store_cvt<T, Sto>::get(shat[kk]), h);
        }
        fft<+1, LOG2L>(a, lds, tw, t);
        PT *row = plane + (int64_t)j * n;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int p = t + kk * TH;
            const int64_t r = s * (int64_t)V + p - half;
            if (p >= half && p < L - half && r < n) {
                const T pw = a[kk].re * a[kk].re + a[kk].im * a[kk].im;
                plane_store<PT>::put(row + r, pw);
            }
        }
    }
}

namespace {

template <int LOG2L, class T, class Sto, class PT>
hipError_t launch_one(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    constexpr int L = 1 << LOG2L;
    const int64_t n_seg = (n + p.V - 1) / p.V;
    const int64_t blocks = n_seg * p.n_chunks;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = (size_t)(L + L / 16) * sizeof(Sto);
    auto k = correlate_valu<LOG2L, T, Sto, PT>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const auto *ws = static_cast<const unsigned char *>(p.ws);
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(L / 16), lds, st, static_cast<const float *>(spec), n,
                       reinterpret_cast<const Sto *>(ws + p.off_bank), reinterpret_cast<const cpx<T> *>(ws + p.off_tw),
                       static_cast<PT *>(plane), p.M, p.V, p.cfg.n_z, p.z_chunk, p.n_chunks);
    return hipGetLastError();
}

template <int LOG2L>
hipError_t dispatch_dtype(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    const int c = p.cfg.compute, pd = p.cfg.plane_dtype;
    if (c == FDAS_FP32 && pd == FDAS_FP32) return launch_one<LOG2L, float, cpx<float>, float>(p, spec, n, plane, st);
    if (c == FDAS_FP32 && pd == FDAS_BF16) return launch_one<LOG2L, float, cpx<float>, __bf16>(p, spec, n, plane, st);
    if (c == FDAS_BF16 && pd == FDAS_FP32) return launch_one<LOG2L, float, bf16c, float>(p, spec, n, plane, st);
    if (c == FDAS_BF16 && pd == FDAS_BF16) return launch_one<LOG2L, float, bf16c, __bf16>(p, spec, n, plane, st);
    if constexpr (LOG2L <= 13) {
        if (c == FDAS_FP64 && pd == FDAS_FP64)
            return launch_one<LOG2L, double, cpx<double>, double>(p, spec, n, plane, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_correlate(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    if (p.cfg.compute == FDAS_FP8E4M3) return launch_correlate_fp8(p, spec, n, plane, st);
    switch (p.log2L) {
        case 10: return dispatch_dtype<10>(p, spec, n, plane, st);
        case 11: return dispatch_dtype<11>(p, spec, n, plane, st);
        case 12: return dispatch_dtype<12>(p, spec, n, plane, st);
        case 13: return dispatch_dtype<13>(p, spec, n, plane, st);
        case 14: return dispatch_dtype<14>(p, spec, n, plane, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdas
