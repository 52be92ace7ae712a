// Overlap-save correlation on the matrix cores: BF16 form, segment L = 8192.
//
// Same plane as the vector-ALU kernel (split the spectrum into overlapping
// windows, transform, multiply by each template's transform, inverse
// transform, keep the central V = L - M outputs; Section "Detailed
// explanation"), with the three DFT stages of every transform executed as
// 16x16x32 bf16 MFMA products (factorisation and operand layout in
// mfma8192.hpp).  One workgroup of 8 waves owns one segment and a chunk of
// templates:
//
//   forward  F1 (DFT32 over n1, input rounded to bf16) -> conj(T2) on VALU ->
//            LDS -> F2 (DFT16 over n2, conj(T1) folded) -> LDS -> F3 (DFT16
//            over n3).  F3 leaves the segment spectrum X[k1, k2, k3] in the
//            registers, exactly in the B-operand layout of the first inverse
//            stage; it is kept as two bf16 pairs (Re, -Im) and (Im, Re) so that
//            each complex product with a template value is two v_dot2_f32_bf16.
//   per template j of the chunk:
//            Y = X * H_j (dot2) -> I1 (DFT16 over k3) -> LDS A -> I2 (DFT16
//            over k2, T1 folded) -> T2 on VALU -> LDS B -> I3 (DFT32 over k1)
//            -> |y|^2 -> plane row j (non-temporal stores).
// Two LDS buffers (A, B) of 8192 bf16 complex words; two barriers per
// template.  The template bank is stored in the lane order of I1 (one
// 16-byte load per lane per MFMA group).
#include "fft_valu.hpp"
#include "internal.hpp"
#include "mfma8192.hpp"
#include "plane_io.hpp"

namespace fdas {
namespace m8k {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

struct alignas(16) Op {
    uint32_t w[4];
};

__device__ __forceinline__ f32x4_t mma(const Op &a, const Op &b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                   c, 0, 0, 0);
}

__device__ __forceinline__ float dot2(uint32_t a, uint32_t b) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), 0.0f,
                                           false);
}

__device__ __forceinline__ Op load_op(const uint32_t *tab, int op, int lane) {
    const uint4 v = reinterpret_cast<const uint4 *>(tab + op * kOpWords)[lane];
    return Op{{v.x, v.y, v.z, v.w}};
}

template <class PT>
__global__ void __launch_bounds__(kThreads, 1)
correlate_mfma8192(const float2 *__restrict__ spec, int64_t n, const uint32_t *__restrict__ bank,
                   const uint32_t *__restrict__ tab, PT *__restrict__ plane, int32_t M, int32_t V, int32_t n_z,
                   int32_t z_chunk, int32_t n_chunks) {
    __shared__ uint32_t bufA[kL];
    __shared__ uint32_t bufB[kL];

    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, c = lane & 15, g = lane >> 4;
    const int chunk = blockIdx.x % n_chunks;
    const int64_t s = blockIdx.x / n_chunks;
    const int j0 = chunk * z_chunk;
    const int j1 = min(j0 + z_chunk, n_z);
    if (j0 >= j1) return;
    const int64_t base = s * (int64_t)V - M / 2;
    const float2 *t2inv = reinterpret_cast<const float2 *>(tab + kNumOps * kOpWords);
    const float2 *t2fwd = t2inv + kT2Count;
    const f32x4_t zero = {0.f, 0.f, 0.f, 0.f};

    // ---------------- forward transform of the segment ----------------
    // F1: groups q < 2 (n2 = 2w + q), column n3 = c, K block kb: n1 = 16 kb + 4 g + p
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int n2 = 2 * w + q;
        Op xb[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int n1 = 16 * kb + 4 * g + p;
                const int64_t idx = base + 256 * n1 + 16 * n2 + c;
                float2 v = make_float2(0.f, 0.f);
                if (idx >= 0 && idx < n) v = spec[idx];
                xb[kb].w[p] = bf16_pack(v.x, v.y);
            }
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            f32x4_t acc = mma(load_op(tab, OP_A32M + mb * 2 + 0, lane), xb[0], zero);
            acc = mma(load_op(tab, OP_A32M + mb * 2 + 1, lane), xb[1], acc);
#pragma unroll
            for (int e2 = 0; e2 < 2; ++e2) {
                const int k1 = 8 * mb + 2 * g + e2;
                const float2 t = t2fwd[(((w * 64 + lane) * 2 + q) * 4 + mb) * 2 + e2];
                const float re = acc[2 * e2], im = acc[2 * e2 + 1];
                bufA[lds_addr(k1, n2, c)] = bf16_pack(re * t.x - im * t.y, re * t.y + im * t.x);
            }
        }
    }
    __syncthreads();
    // F2: groups q < 4: n3 = 4 (w % 4) + q, column k1 = 16 (w / 4) + c, K: n2 = 4 g + p
    {
        const int k1 = 16 * (w >> 2) + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int n3 = 4 * (w & 3) + q;
            Op b;
#pragma unroll
            for (int p = 0; p < 4; ++p) b.w[p] = bufA[lds_addr(k1, 4 * g + p, n3)];
            const f32x4_t dre = mma(load_op(tab, OP_AF2M + 2 * n3, lane), b, zero);
            const f32x4_t dim = mma(load_op(tab, OP_AF2M + 2 * n3 + 1, lane), b, zero);
#pragma unroll
            for (int e = 0; e < 4; ++e) bufB[lds_addr(k1, 4 * g + e, n3)] = bf16_pack(dre[e], dim[e]);
        }
    }
    __syncthreads();
    // F3: groups q < 4: k1 = 4 w + q, column k2 = c, K: n3 = 4 g + p
    uint32_t sA[4][4], sB[4][4];   // (Re, -Im) and (Im, Re) of X[k1, k2 = c, k3 = 4 g + p]
    {
        const Op a16re = load_op(tab, OP_A16M, lane), a16im = load_op(tab, OP_A16M + 1, lane);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Op b;
#pragma unroll
            for (int p = 0; p < 4; ++p) b.w[p] = bufB[lds_addr(4 * w + q, c, 4 * g + p)];
            const f32x4_t dre = mma(a16re, b, zero);
            const f32x4_t dim = mma(a16im, b, zero);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                sA[q][p] = bf16_pack(dre[p], -dim[p]);
                sB[q][p] = bf16_pack(dim[p], dre[p]);
            }
        }
    }

    // ---------------- persistent inverse operators ----------------
    const Op a16re = load_op(tab, OP_A16P, lane), a16im = load_op(tab, OP_A16P + 1, lane);
    Op a2re[4], a2im[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n3 = 4 * (w & 3) + q;
        a2re[q] = load_op(tab, OP_A2P + 2 * n3, lane);
        a2im[q] = load_op(tab, OP_A2P + 2 * n3 + 1, lane);
    }
    Op a32[4][2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        a32[mb][0] = load_op(tab, OP_A32P + mb * 2, lane);
        a32[mb][1] = load_op(tab, OP_A32P + mb * 2 + 1, lane);
    }
    float2 t2[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) t2[q][e] = t2inv[((w * 64 + lane) * 4 + q) * 4 + e];

    const int half = M / 2;
    const int64_t seg0 = s * (int64_t)V - half;   // plane column of time index n is seg0 + n
    const bool full = seg0 + (kL - half) <= n;    // every kept output lies inside the plane

    for (int j = j0; j < j1; ++j) {
        // I1: Y = X * H_j, DFT16 over k3; groups q < 4: k1 = 4 w + q, column k2 = c
        const uint4 *hb = reinterpret_cast<const uint4 *>(bank + (size_t)j * kL) + (w * 4) * 64 + lane;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 h = hb[q * 64];
            const uint32_t hw[4] = {h.x, h.y, h.z, h.w};
            Op b;
#pragma unroll
            for (int p = 0; p < 4; ++p) b.w[p] = bf16_pack(dot2(sA[q][p], hw[p]), dot2(sB[q][p], hw[p]));
            const f32x4_t dre = mma(a16re, b, zero);
            const f32x4_t dim = mma(a16im, b, zero);
#pragma unroll
            for (int e = 0; e < 4; ++e) bufA[lds_addr(4 * w + q, c, 4 * g + e)] = bf16_pack(dre[e], dim[e]);
        }
        __syncthreads();
        // I2: DFT16 over k2 with T1 folded; groups q < 4: n3 = 4 (w % 4) + q, column k1 = 16 (w / 4) + c
        {
            const int k1 = 16 * (w >> 2) + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n3 = 4 * (w & 3) + q;
                Op b;
#pragma unroll
                for (int p = 0; p < 4; ++p) b.w[p] = bufA[lds_addr(k1, 4 * g + p, n3)];
                const f32x4_t dre = mma(a2re[q], b, zero);
                const f32x4_t dim = mma(a2im[q], b, zero);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float2 t = t2[q][e];
                    bufB[lds_addr(k1, 4 * g + e, n3)] =
                        bf16_pack(dre[e] * t.x - dim[e] * t.y, dre[e] * t.y + dim[e] * t.x);
                }
            }
        }
        __syncthreads();
        // I3: DFT32 over k1; groups q < 2: n2 = 2 w + q, column n3 = c
        PT *row = plane + (int64_t)j * n;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int n2 = 2 * w + q;
            Op b[2];
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int p = 0; p < 4; ++p) b[kb].w[p] = bufB[lds_addr(16 * kb + 4 * g + p, n2, c)];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                f32x4_t acc = mma(a32[mb][0], b[0], zero);
                acc = mma(a32[mb][1], b[1], acc);
#pragma unroll
                for (int e2 = 0; e2 < 2; ++e2) {
                    const int n1 = 8 * mb + 2 * g + e2;
                    const int t = 256 * n1 + 16 * n2 + c;          // time index in the segment
                    const float pw = acc[2 * e2] * acc[2 * e2] + acc[2 * e2 + 1] * acc[2 * e2 + 1];
                    const int64_t col = seg0 + t;
                    if (t >= half && t < kL - half && (full || col < n)) plane_store<PT>::put(row + col, pw);
                }
            }
        }
    }
}

namespace {
template <class PT>
hipError_t launch(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    const int64_t n_seg = (n + p.V - 1) / p.V;
    const int64_t blocks = n_seg * p.n_chunks;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const auto *ws = static_cast<const unsigned char *>(p.ws);
    hipLaunchKernelGGL(correlate_mfma8192<PT>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                       static_cast<const float2 *>(spec), n, reinterpret_cast<const uint32_t *>(ws + p.off_bank),
                       reinterpret_cast<const uint32_t *>(ws + p.off_tab), static_cast<PT *>(plane), p.M, p.V,
                       p.cfg.n_z, p.z_chunk, p.n_chunks);
    return hipGetLastError();
}
}  // namespace

}  // namespace m8k

hipError_t launch_correlate_mfma(const fdas_plan_s &p, const void *spec, int64_t n, void *plane, hipStream_t st) {
    if (p.L != m8k::kL || p.cfg.compute != FDAS_BF16) return hipErrorInvalidValue;
    if (p.cfg.plane_dtype == FDAS_BF16) return m8k::launch<__bf16>(p, spec, n, plane, st);
    if (p.cfg.plane_dtype == FDAS_FP32) return m8k::launch<float>(p, spec, n, plane, st);
    return hipErrorInvalidValue;
}

}  // namespace fdas
