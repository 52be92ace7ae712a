// Overlap-save correlation in the FP8 (OCP e4m3) storage form.
//
// The same plane as the other forms (Section "Detailed explanation"), with
// the precision one step below bfloat16 (Section "Updating the pipeline to
// bfloat16" argues for narrower storage with wide accumulation; FP8 is the
// next format gfx950 stores natively).  The window is read in FP32 (the
// paper keeps its real FFT in single precision); every transform stage that
// goes through LDS, the segment spectrum kept across the template chunk and
// the template bank are e4m3 with power-of-two scales (fft_fp8.hpp); all
// arithmetic is FP32.  Structure as the vector-ALU kernel: one workgroup owns
// a segment and a chunk of templates, 16 points per thread, Stockham passes.
#include "fft_fp8.hpp"
#include "internal.hpp"
#include "plane_io.hpp"

namespace fdas {

template <int LOG2L, class PT>
__global__ void __launch_bounds__((1 << LOG2L) / 16)
correlate_valu_fp8(const float *__restrict__ spec, int64_t n, const fp8c *__restrict__ bank,
                   const int32_t *__restrict__ texp, const cpx<float> *__restrict__ tw, PT *__restrict__ plane,
                   int32_t M, int32_t V, int32_t n_z, int32_t z_chunk, int32_t n_chunks) {
    constexpr int L = 1 << LOG2L;
    constexpr int TH = L / 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fp8c *lds = reinterpret_cast<fp8c *>(smem_raw);
    __shared__ unsigned int slots[2];

    const int t = threadIdx.x;
    const int chunk = blockIdx.x % n_chunks;
    const int64_t s = blockIdx.x / n_chunks;
    const int j0 = chunk * z_chunk;
    const int j1 = min(j0 + z_chunk, n_z);
    if (j0 >= j1) return;
    const int64_t base = s * (int64_t)V - M / 2;
    if (t == 0) slots[0] = slots[1] = 0u;
    int slot = 0;

    cpx<float> a[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        const int64_t idx = base + t + kk * TH;
        if (idx >= 0 && idx < n) {
            const float2 v = reinterpret_cast<const float2 *>(spec)[idx];
            a[kk] = {v.x, v.y};
        } else {
            a[kk] = {0.0f, 0.0f};
        }
    }
    __syncthreads();   // slots cleared
    fft_fp8<-1, LOG2L>(a, lds, tw, t, slots, slot);

    // segment spectrum as scaled e4m3
    float m = 0.0f;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) m = fmaxf(m, cmax_abs(a[kk]));
    const float sS = fp8_scale_for(block_amax(m, slots, slot));
    const float invS = 1.0f / sS;
    uint16_t shat[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) shat[kk] = fp8_pack(a[kk].re * sS, a[kk].im * sS);

    const int half = M / 2;
    for (int j = j0; j < j1; ++j) {
        const fp8c *hb = bank + (int64_t)j * L;
        const float sc = invS * ldexpf(1.0f, -texp[j]);   // undo both power-of-two scales
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const cpx<float> y = cmul(fp8_unpack(shat[kk]), fp8_unpack(hb[t + kk * TH].bits));
            a[kk] = {y.re * sc, y.im * sc};
        }
        fft_fp8<+1, LOG2L>(a, lds, tw, t, slots, slot);
        PT *row = plane + (int64_t)j * n;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int p = t + kk * TH;
            const int64_t r = s * (int64_t)V + p - half;
            if (p >= half && p < L - half && r < n) {
                const float pw = a[kk].re * a[kk].re + a[kk].im * a[kk].im;
                plane_store<PT>::put(row + r, pw);
            }
        }
    }
}

// Template bank in e4m3: per template j the largest power of two 2^t_j that
// keeps every |re| / |im| of the FP32 spectrum <= 448; bank = e4m3(H 2^t_j),
// texp[j] = t_j.  Grid: one workgroup of 256 threads per template.
__global__ void __launch_bounds__(256) k_fp8_bank(const cpx<float> *h32, fp8c *bank, int32_t *texp, int32_t L) {
    __shared__ float red[256];
    const int j = blockIdx.x;
    const cpx<float> *h = h32 + (int64_t)j * L;
    float m = 0.0f;
    for (int k = threadIdx.x; k < L; k += 256) m = fmaxf(m, cmax_abs(h[k]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const float sc = fp8_scale_for(red[0]);
    if (threadIdx.x == 0) texp[j] = ilogbf(sc);
    for (int k = threadIdx.x; k < L; k += 256) bank[(int64_t)j * L + k] = fp8c{fp8_pack(h[k].re * sc, h[k].im * sc)};
}

namespace {

template <int LOG2L, class PT>
hipError_t launch_fp8(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    constexpr int L = 1 << LOG2L;
    const int64_t n_seg = (n + p.V - 1) / p.V;
    const int64_t blocks = n_seg * p.n_chunks;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = (size_t)(L + L / 16) * sizeof(fp8c);
    const auto *ws = static_cast<const unsigned char *>(p.ws);
    hipLaunchKernelGGL((correlate_valu_fp8<LOG2L, PT>), dim3((unsigned)blocks), dim3(L / 16), lds, st,
                       static_cast<const float *>(spec), n, reinterpret_cast<const fp8c *>(ws + p.off_bank),
                       reinterpret_cast<const int32_t *>(ws + p.off_tab + fp8_staging_bytes(p)),
                       reinterpret_cast<const cpx<float> *>(ws + p.off_tw), static_cast<PT *>(plane), p.M, p.V,
                       p.cfg.n_z, p.z_chunk, p.n_chunks);
    return hipGetLastError();
}

template <int LOG2L>
hipError_t dispatch_fp8(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    if (p.cfg.plane_dtype == FDAS_FP32) return launch_fp8<LOG2L, float>(p, spec, n, plane, st);
    if (p.cfg.plane_dtype == FDAS_BF16) return launch_fp8<LOG2L, __bf16>(p, spec, n, plane, st);
    return hipErrorInvalidValue;
}

}  // namespace

size_t fp8_staging_bytes(const fdas_plan_s &p) { return (size_t)p.cfg.n_z * p.L * sizeof(cpx<float>); }

hipError_t launch_fp8_bank(const fdas_plan_s &p, hipStream_t st) {
    unsigned char *ws = static_cast<unsigned char *>(p.ws);
    hipLaunchKernelGGL(k_fp8_bank, dim3((unsigned)p.cfg.n_z), dim3(256), 0, st,
                       reinterpret_cast<const cpx<float> *>(ws + p.off_tab), reinterpret_cast<fp8c *>(ws + p.off_bank),
                       reinterpret_cast<int32_t *>(ws + p.off_tab + fp8_staging_bytes(p)), p.L);
    return hipGetLastError();
}

hipError_t launch_correlate_fp8(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    switch (p.log2L) {
        case 10: return dispatch_fp8<10>(p, spec, n, plane, st);
        case 11: return dispatch_fp8<11>(p, spec, n, plane, st);
        case 12: return dispatch_fp8<12>(p, spec, n, plane, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdas
