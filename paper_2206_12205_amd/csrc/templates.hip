// Template bank and twiddle table, built on the GPU in double precision.
//
// The paper generates its templates in a higher precision and converts them
// to the reduced one with a GPU kernel (Section "Template conversion"; the
// bfloat16 conversion statistics are Table 1).  Here:
//   taps      g_j[m] = conj(A(m - z_j/2, z_j)),  m in [-M/2, M/2)   (FP64);
//             with a jerk w: conj(A(m - z_j/2 - w/6, z_j, w)) (response.hpp)
//   norm      g_j /= ||g_j||_2                                       (FP64)
//   spectrum  H_j[k] = (1/L) sum_m g_j[m] exp(-2 pi i k m / L),  k in [0, L)
//             i.e. the length-L DFT of the circularly placed taps h[m mod L],
//             summed directly over the M nonzero taps in FP64, with the 1/L
//             of the inverse transform folded in
//   cast      FP32: one round-to-nearest-even cast of the FP64 value;
//             BF16: the FP32 value rounded again to bfloat16 (the paper
//             converts single-precision templates to bfloat16);
//             FP64: stored as is.
//   twiddles  tw[e] = exp(-2 pi i e / L), e in [0, L), FP64 -> compute type.
#include "fft_valu.hpp"
#include "internal.hpp"
#include "mfma4096.hpp"
#include "mfma8192.hpp"
#include "response.hpp"

namespace fdas {

__global__ void k_taps(cd *taps, int32_t n_z, int32_t M, double z_min, double z_step) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_z * M) return;
    const int j = (int)(i / M);
    const int m = (int)(i % M) - M / 2;
    const double z = z_min + z_step * j;
    taps[i] = conj(response((double)m - 0.5 * z, z));
}

// Taps of a jerk search plane: g_j[m] = conj(A(m - z_j/2 - w/6, z_j, w)),
// m - z_j/2 - w/6 being the offset from the mean frequency r0 + z/2 + w/6.
__global__ void __launch_bounds__(256) k_taps_jerk(cd *taps, int32_t n_z, int32_t M, double z_min, double z_step,
                                                   double w) {
    // one wave per tap: lanes take the quadrature panels in turn, then a
    // butterfly sum over the wave (a fixed order, so the bank is reproducible)
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= (int64_t)n_z * M) return;   // uniform over the wave
    const int j = (int)(i / M);
    const int m = (int)(i % M) - M / 2;
    const double z = z_min + z_step * j;
    cd s = response_jerk_panels((double)m - 0.5 * z - w / 6.0, z, w, lane, 64);
    for (int off = 32; off > 0; off >>= 1) {
        s.re += __shfl_xor(s.re, off);
        s.im += __shfl_xor(s.im, off);
    }
    if (lane == 0) taps[i] = conj(s);
}

// One workgroup per template: l2 norm by a fixed-order tree reduction.
__global__ void __launch_bounds__(256) k_normalise(cd *taps, int32_t M) {
    __shared__ double red[256];
    cd *g = taps + (int64_t)blockIdx.x * M;
    double s = 0.0;
    for (int i = threadIdx.x; i < M; i += 256) s += g[i].re * g[i].re + g[i].im * g[i].im;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double inv = 1.0 / sqrt(red[0]);
    for (int i = threadIdx.x; i < M; i += 256) g[i] = inv * g[i];
}

template <class B>
__device__ __forceinline__ B bank_cast(cd v);
template <>
__device__ __forceinline__ cpx<float> bank_cast<cpx<float>>(cd v) { return {(float)v.re, (float)v.im}; }
template <>
__device__ __forceinline__ cpx<double> bank_cast<cpx<double>>(cd v) { return {v.re, v.im}; }
template <>
__device__ __forceinline__ bf16c bank_cast<bf16c>(cd v) { return {bf16_pack((float)v.re, (float)v.im)}; }

// Grid: (L / 256, n_z); taps of template j staged in LDS.
// Position of frequency bin k of template j in the bank: natural order (0),
// or the lane order of the matrix-core kernels for L = 8192 (1) / 4096 (2).
__device__ __forceinline__ int64_t bank_pos(int j, int k, int L, int order) {
    if (order == 0) return (int64_t)j * L + k;
    if (order == 2) return (int64_t)j * L + m4k::bank_pos_of(k);
    const int k1 = k & 31, k2 = (k >> 5) & 15, k3 = k >> 9;
    const int wave = k1 >> 2, q = k1 & 3, lane = k2 + 16 * (k3 >> 2), p = k3 & 3;
    return (int64_t)j * L + (((wave * 4 + q) * 64 + lane) * 4 + p);
}

// Roots exp(-2 pi i e / L) from two LDS tables, e = 64 a + b: the high
// table exp(-2 pi i 64 a / L) (L / 64 entries) times the low one
// exp(-2 pi i b / L) (64 entries), each entry one FP64 sincospi, so a term
// costs one complex FP64 product instead of a sincospi.  L is a power of two
// (>= 1024), so e = m k mod L is a mask and steps by k from one tap to the
// next.
constexpr int kRootLo = 64;

static size_t spectrum_lds_bytes(int32_t M, int32_t L) { return (size_t)(M + kRootLo + L / kRootLo) * sizeof(cd); }

template <class B>
__global__ void __launch_bounds__(256) k_spectrum(const cd *taps, B *bank, int32_t M, int32_t L, int order) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cd *g = reinterpret_cast<cd *>(smem_raw);
    cd *wlo = g + M;
    cd *whi = wlo + kRootLo;
    const int j = blockIdx.y;
    for (int i = threadIdx.x; i < M; i += 256) g[i] = taps[(int64_t)j * M + i];
    for (int i = threadIdx.x; i < kRootLo; i += 256) {
        double sn, cs;
        sincospi(-2.0 * (double)i / (double)L, &sn, &cs);
        wlo[i] = cd{cs, sn};
    }
    for (int i = threadIdx.x; i < L / kRootLo; i += 256) {
        double sn, cs;
        sincospi(-2.0 * (double)(kRootLo * i) / (double)L, &sn, &cs);
        whi[i] = cd{cs, sn};
    }
    __syncthreads();
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= L) return;
    const uint32_t mask = (uint32_t)L - 1u;
    uint32_t e = (uint32_t)(((int64_t)(-(M / 2)) * (int64_t)k) & (int64_t)mask);   // m = -M/2
    double re = 0.0, im = 0.0;
    for (int i = 0; i < M; ++i) {
        const cd a = whi[e / kRootLo], b = wlo[e % kRootLo];
        const double cs = a.re * b.re - a.im * b.im, sn = a.re * b.im + a.im * b.re;
        re += g[i].re * cs - g[i].im * sn;
        im += g[i].re * sn + g[i].im * cs;
        e = (e + (uint32_t)k) & mask;
    }
    const double invL = 1.0 / (double)L;
    bank[bank_pos(j, k, L, order)] = bank_cast<B>(cd{re * invL, im * invL});
}

// exp(s 2 pi i m / N) for integer m, FP64.
__device__ __forceinline__ cd unit_root(int64_t m, int64_t N, int s) {
    int64_t r = m % N;
    if (r < 0) r += N;
    double sn, cs;
    sincospi(2.0 * (double)r / (double)N, &sn, &cs);
    return {cs, s > 0 ? sn : -sn};
}

// Operators and per-lane twiddles of the length-8192 matrix-core kernel.
// One thread per (op, lane) or per twiddle slot; see mfma8192.hpp.
__global__ void k_m8k_tables(uint32_t *tab) {
    using namespace m8k;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_op_threads = kNumOps * 64;
    if (t < n_op_threads) {
        const int op = t / 64, lane = t % 64, c = lane & 15, g = lane >> 4;
        uint32_t w[4];
        for (int e = 0; e < 8; e += 2) {
            float v[2];
            for (int h = 0; h < 2; ++h) {
                const int el = e + h;
                const int part_in = el & 1;
                cd a;
                int part_out;
                if (op >= OP_A32P && op < OP_AF2M) {          // DFT32 (inverse or forward)
                    const int rel = (op - (op < OP_A32M ? OP_A32P : OP_A32M));
                    const int mb = rel >> 1, kb = rel & 1;
                    const int n1 = 8 * mb + (c >> 1);
                    part_out = c & 1;
                    const int k1 = 16 * kb + 4 * g + (el >> 1);
                    a = unit_root((int64_t)n1 * k1, 32, op < OP_A32M ? +1 : -1);
                } else {                                       // DFT16 variants
                    const int row = c, pin = 4 * g + (el >> 1);
                    int imrows;
                    if (op < OP_A2P) {                         // inverse DFT16
                        imrows = op - OP_A16P;
                        a = unit_root((int64_t)row * pin, 16, +1);
                    } else if (op < OP_A32P) {                 // inverse DFT16 with T1(k2 = pin; n3)
                        const int n3 = (op - OP_A2P) >> 1;
                        imrows = (op - OP_A2P) & 1;
                        a = unit_root((int64_t)16 * row * pin + (int64_t)n3 * pin, 256, +1);
                    } else if (op < OP_A16M) {                 // forward DFT16 with conj T1(k2 = row; n3)
                        const int n3 = (op - OP_AF2M) >> 1;
                        imrows = (op - OP_AF2M) & 1;
                        a = unit_root((int64_t)16 * row * pin + (int64_t)n3 * row, 256, -1);
                    } else {                                   // forward DFT16
                        imrows = op - OP_A16M;
                        a = unit_root((int64_t)row * pin, 16, -1);
                    }
                    part_out = imrows;
                }
                double val;
                if (part_out == 0) val = part_in ? -a.im : a.re;
                else val = part_in ? a.re : a.im;
                v[h] = (float)val;
            }
            w[e >> 1] = bf16_pack(v[0], v[1]);
        }
        for (int i = 0; i < 4; ++i) tab[op * kOpWords + lane * 4 + i] = w[i];
        return;
    }
    const int u = t - n_op_threads;
    float2 *tw = reinterpret_cast<float2 *>(tab + kNumOps * kOpWords);
    if (u < kT2Count) {                                        // inverse T2: [wave][lane][q][e]
        const int e = u & 3, q = (u >> 2) & 3, lane = (u >> 4) & 63, wave = u >> 10;
        const int c = lane & 15, g = lane >> 4;
        const int k1 = 16 * (wave >> 2) + c, n2 = 4 * g + e, n3 = 4 * (wave & 3) + q;
        const cd r = unit_root((int64_t)(16 * n2 + n3) * k1, kL, +1);
        tw[u] = make_float2((float)r.re, (float)r.im);
        return;
    }
    const int v = u - kT2Count;
    if (v < kT2FCount) {                                       // forward conj T2: [wave][lane][q][mb][e2]
        const int e2 = v & 1, mb = (v >> 1) & 3, q = (v >> 3) & 1, lane = (v >> 4) & 63, wave = v >> 10;
        const int c = lane & 15, g = lane >> 4;
        const int n2 = 2 * wave + q, n3 = c, k1 = 8 * mb + 2 * g + e2;
        const cd r = unit_root((int64_t)(16 * n2 + n3) * k1, kL, -1);
        tw[kT2Count + v] = make_float2((float)r.re, (float)r.im);
    }
}

// Stage operators of the length-4096 matrix-core kernel (mfma4096.hpp), one
// thread per (op, lane).
__global__ void k_m4k_tables(uint32_t *tab) {
    using namespace m4k;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kNumOps * 64) return;
    const int op = t / 64, lane = t % 64, c = lane & 15, g = lane >> 4;
    const int op0 = op & ~31, G = (op & 31) >> 1, part_out = op & 1;
    uint32_t w[4];
    for (int e = 0; e < 8; e += 2) {
        float v[2];
        for (int h = 0; h < 2; ++h) {
            const int el = e + h, part_in = el & 1;
            const cd a = unit_root(op_exponent(op0, G, c, 4 * g + (el >> 1)), kL, +1);
            const double val = part_out == 0 ? (part_in ? -a.im : a.re) : (part_in ? a.re : a.im);
            v[h] = (float)val;
        }
        w[e >> 1] = bf16_pack(v[0], v[1]);
    }
    for (int i = 0; i < 4; ++i) tab[op * kOpWords + lane * 4 + i] = w[i];
}

template <class R>
__global__ void k_twiddles(cpx<R> *tw, int32_t L) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= L) return;
    double sn, cs;
    sincospi(-2.0 * (double)e / (double)L, &sn, &cs);
    tw[e] = {(R)cs, (R)sn};
}

hipError_t launch_make_templates(const fdas_plan_s &p, hipStream_t st, double w) {
    unsigned char *ws = static_cast<unsigned char *>(p.ws);
    cd *taps = reinterpret_cast<cd *>(ws + p.off_taps);
    const int64_t nt = (int64_t)p.cfg.n_z * p.M;
    if (w == 0.0)
        hipLaunchKernelGGL(k_taps, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, taps, p.cfg.n_z, p.M,
                           p.cfg.z_min, p.cfg.z_step);
    else
        hipLaunchKernelGGL(k_taps_jerk, dim3((unsigned)((nt + 3) / 4)), dim3(256), 0, st, taps, p.cfg.n_z, p.M,
                           p.cfg.z_min, p.cfg.z_step, w);   // four taps (waves) per workgroup
    hipLaunchKernelGGL(k_normalise, dim3(p.cfg.n_z), dim3(256), 0, st, taps, p.M);
    const dim3 grid((unsigned)((p.L + 255) / 256), (unsigned)p.cfg.n_z);
    const size_t lds = spectrum_lds_bytes(p.M, p.L);
    void *bank = ws + p.off_bank;
    hipError_t e = hipSuccess;
    switch (p.cfg.compute) {
        case FDAS_FP32: e = hipFuncSetAttribute((const void *)k_spectrum<cpx<float>>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
        case FDAS_BF16: e = hipFuncSetAttribute((const void *)k_spectrum<bf16c>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
        case FDAS_FP64: e = hipFuncSetAttribute((const void *)k_spectrum<cpx<double>>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
        case FDAS_FP8E4M3: e = hipFuncSetAttribute((const void *)k_spectrum<cpx<float>>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    switch (p.cfg.compute) {
        case FDAS_FP32:
            hipLaunchKernelGGL(k_spectrum<cpx<float>>, grid, dim3(256), lds, st, taps,
                               static_cast<cpx<float> *>(bank), p.M, p.L, 0);
            hipLaunchKernelGGL(k_twiddles<float>, dim3((p.L + 255) / 256), dim3(256), 0, st,
                               reinterpret_cast<cpx<float> *>(ws + p.off_tw), p.L);
            break;
        case FDAS_BF16:
            hipLaunchKernelGGL(k_spectrum<bf16c>, grid, dim3(256), lds, st, taps, static_cast<bf16c *>(bank), p.M,
                               p.L, !p.mfma ? 0 : (p.L == m8k::kL ? 1 : 2));
            if (p.mfma && p.L == m8k::kL) {
                const int nthreads = m8k::kNumOps * 64 + m8k::kT2Count + m8k::kT2FCount;
                hipLaunchKernelGGL(k_m8k_tables, dim3((nthreads + 255) / 256), dim3(256), 0, st,
                                   reinterpret_cast<uint32_t *>(ws + p.off_tab));
            } else if (p.mfma) {
                const int nthreads = m4k::kNumOps * 64;
                hipLaunchKernelGGL(k_m4k_tables, dim3((nthreads + 255) / 256), dim3(256), 0, st,
                                   reinterpret_cast<uint32_t *>(ws + p.off_tab));
            }
            hipLaunchKernelGGL(k_twiddles<float>, dim3((p.L + 255) / 256), dim3(256), 0, st,
                               reinterpret_cast<cpx<float> *>(ws + p.off_tw), p.L);
            break;
        case FDAS_FP8E4M3:
            // FP32 spectrum into the staging area, then per-template scaled e4m3
            hipLaunchKernelGGL(k_spectrum<cpx<float>>, grid, dim3(256), lds, st, taps,
                               reinterpret_cast<cpx<float> *>(ws + p.off_tab), p.M, p.L, 0);
            e = launch_fp8_bank(p, st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_twiddles<float>, dim3((p.L + 255) / 256), dim3(256), 0, st,
                               reinterpret_cast<cpx<float> *>(ws + p.off_tw), p.L);
            break;
        case FDAS_FP64:
            hipLaunchKernelGGL(k_spectrum<cpx<double>>, grid, dim3(256), lds, st, taps,
                               static_cast<cpx<double> *>(bank), p.M, p.L, 0);
            hipLaunchKernelGGL(k_twiddles<double>, dim3((p.L + 255) / 256), dim3(256), 0, st,
                               reinterpret_cast<cpx<double> *>(ws + p.off_tw), p.L);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdas
