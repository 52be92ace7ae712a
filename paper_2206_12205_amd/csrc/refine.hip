// Candidate refinement: matched-filter power at continuous (r, z) and its
// gradient, with optional gradient ascent.
//
// The plane samples the matched-filter power on integer r and a z grid; the
// quantisation in both axes moves peaks into adjacent bins (Section
// "Peakfinding methodology").  Refinement evaluates the same matched filter
// at continuous (r, z) from a window of K spectral bins around r,
//
//   F(r, z) = sum_{k = floor(r) - K/2 + 1}^{floor(r) + K/2} X[k] conj(A(r - z/2 - k, z)),
//   P = |F|^2,
//   dP/dr = 2 Re(conj(F) sum X[k] conj(A_q)),
//   dP/dz = 2 Re(conj(F) sum X[k] conj(A_z - A_q / 2)),
//
// with A(q, z) = int_0^1 exp(i pi (2 q u + z u^2)) du (mean-frequency
// convention, X = 0 outside [0, N)).  The derivatives follow from integrating
// d/du exp(i phi) and d/du (u exp(i phi)), phi = pi (2 q u + z u^2), by parts:
//   M1 = int u e^{i phi} = (E1 - 1 - 2 pi i q A) / (2 pi i z)
//   M2 = int u^2 e^{i phi} = (E1 - A - 2 pi i q M1) / (2 pi i z),  E1 = e^{i pi (2q + z)},
//   A_q = 2 pi i M1,  A_z = i pi M2,
// used for |z| >= kClosedFormZ; below that the three moments come from
// composite 16-point Gauss-Legendre quadrature (panels resolving every half
// turn).  The closed form divides by z twice: its numerators are O(z) with
// absolute errors near eps (1 + 2 pi |q| |A|), so M2 carries about
// eps 2 pi |q| / (2 pi z)^2, 2e-12 at z = 0.05 and |q| = 16 taps out -- far
// inside the refinement's bars -- while the quadrature costs about
// 32 (|q| + |z|) evaluations of exp(i phi) per tap, which made the few
// candidates near z = 0 set the launch time.
//
// Ascent step (the paper prints none): a Newton step on the analytic
// curvature of an isolated peak, r += s_r 3 / (2 pi^2 P) dP/dr and
// z += s_z 90 / (pi^2 P) dP/dz.
//
// One segment of 32 lanes per candidate when taps <= 32 (two candidates per
// wave), else the whole wave; lane i of the segment holds tap i; the three
// sums are reduced by an XOR butterfly inside the segment (fixed order, the
// same on every lane), so every lane sees the same (r, z) trajectory.
// Everything is FP64: a bin index near 4e6 has an FP32 spacing of half a
// bin.
#include "internal.hpp"
#include "response.hpp"

namespace fdas {

constexpr double kClosedFormZ = 0.05;

// A, A_q, A_z at (q, z).
__device__ void response_d(double q, double z, cd &A, cd &Aq, cd &Az) {
    const double twopi = 2.0 * M_PI;
    if (fabs(z) >= kClosedFormZ) {
        A = response(q, z);
        const cd E1 = expipi(2.0 * q + z);
        const cd tq = {-twopi * q * A.im, twopi * q * A.re};            // 2 pi i q A
        const cd inv2piz = {0.0, -1.0 / (twopi * z)};                  // 1 / (2 pi i z)
        const cd M1 = (E1 - mk(1.0, 0.0) - tq) * inv2piz;
        const cd tq1 = {-twopi * q * M1.im, twopi * q * M1.re};        // 2 pi i q M1
        const cd M2 = (E1 - A - tq1) * inv2piz;
        Aq = {-twopi * M1.im, twopi * M1.re};
        Az = {-M_PI * M2.im, M_PI * M2.re};
        return;
    }
    const int npan = (int)ceil(2.0 * (fabs(q) + fabs(z))) + 2;
    cd m0 = {0, 0}, m1 = {0, 0}, m2 = {0, 0};
    for (int pn = 0; pn < npan; ++pn) {
        for (int i = 0; i < 16; ++i) {
            const double u = (pn + kGLx[i]) / npan;
            const double wt = kGLw[i] / npan;
            const cd e = expipi(2.0 * q * u + z * u * u);
            m0 = m0 + wt * e;
            m1 = m1 + (wt * u) * e;
            m2 = m2 + (wt * u * u) * e;
        }
    }
    A = m0;
    Aq = {-twopi * m1.im, twopi * m1.re};
    Az = {-M_PI * m2.im, M_PI * m2.re};
}

// Sum over the lanes of a segment of `width` (32 or 64) lanes.
__device__ __forceinline__ double seg_sum(double v, int width) {
    if (width == 64) v += __shfl_xor(v, 32, 64);
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct RefineOut {
    double P, dPr, dPz;
};

// Every lane of the segment (width lanes) returns the same values.
__device__ RefineOut eval_point(const float2 *spec, int64_t n, double r, double z, int taps, int lane, int width) {
    cd F = {0, 0}, Fr = {0, 0}, Fz = {0, 0};
    if (lane < taps) {
        const int64_t k = (int64_t)floor(r) - taps / 2 + 1 + lane;
        if (k >= 0 && k < n) {
            const float2 xv = spec[k];
            const cd x = {(double)xv.x, (double)xv.y};
            cd A, Aq, Az;
            response_d(r - 0.5 * z - (double)k, z, A, Aq, Az);
            F = x * conj(A);
            Fr = x * conj(Aq);
            Fz = x * conj(Az - 0.5 * Aq);
        }
    }
    F = {seg_sum(F.re, width), seg_sum(F.im, width)};
    Fr = {seg_sum(Fr.re, width), seg_sum(Fr.im, width)};
    Fz = {seg_sum(Fz.re, width), seg_sum(Fz.im, width)};
    RefineOut o;
    o.P = F.re * F.re + F.im * F.im;
    o.dPr = 2.0 * (F.re * Fr.re + F.im * Fr.im);
    o.dPz = 2.0 * (F.re * Fz.re + F.im * Fz.im);
    return o;
}

__global__ void __launch_bounds__(64) k_refine(const float2 *spec, int64_t n, int32_t n_cand, double *r, double *z,
                                               double *power, double *dp_dr, double *dp_dz, int32_t taps,
                                               int32_t n_steps, double s_r, double s_z) {
    const int width = taps <= 32 ? 32 : 64;   // lanes per candidate
    const int cand = blockIdx.x * (64 / width) + (int)threadIdx.x / width;
    if (cand >= n_cand) return;   // a whole segment: its shuffles stay inside it
    const int lane = (int)threadIdx.x % width;
    double rr = r[cand], zz = z[cand];
    const double pi2 = M_PI * M_PI;
    for (int it = 0; it < n_steps; ++it) {
        const RefineOut o = eval_point(spec, n, rr, zz, taps, lane, width);
        const double Ps = fmax(o.P, 1e-30);
        rr += s_r * 3.0 / (2.0 * pi2 * Ps) * o.dPr;
        zz += s_z * 90.0 / (pi2 * Ps) * o.dPz;
    }
    const RefineOut o = eval_point(spec, n, rr, zz, taps, lane, width);
    if (lane == 0) {
        r[cand] = rr;
        z[cand] = zz;
        if (power) power[cand] = o.P;
        if (dp_dr) dp_dr[cand] = o.dPr;
        if (dp_dz) dp_dz[cand] = o.dPz;
    }
}

// Vector-Jacobian product of P(r, z): grad_r = g dP/dr, grad_z = g dP/dz.
__global__ void __launch_bounds__(64) k_refine_backward(const float2 *spec, int64_t n, int32_t n_cand, const double *r,
                                                        const double *z, const double *grad_p, double *grad_r,
                                                        double *grad_z, int32_t taps) {
    const int width = taps <= 32 ? 32 : 64;
    const int cand = blockIdx.x * (64 / width) + (int)threadIdx.x / width;
    if (cand >= n_cand) return;
    const int lane = (int)threadIdx.x % width;
    const RefineOut o = eval_point(spec, n, r[cand], z[cand], taps, lane, width);
    if (lane == 0) {
        const double g = grad_p[cand];
        grad_r[cand] = g * o.dPr;
        grad_z[cand] = g * o.dPz;
    }
}

hipError_t launch_refine(const void *spec, int64_t n, int32_t n_cand, double *r, double *z, double *power,
                         double *dp_dr, double *dp_dz, int32_t taps, int32_t n_steps, double s_r, double s_z,
                         hipStream_t st) {
    if (n_cand == 0) return hipSuccess;
    const int per = taps <= 32 ? 2 : 1;   // candidates per wave
    hipLaunchKernelGGL(k_refine, dim3((unsigned)((n_cand + per - 1) / per)), dim3(64), 0, st,
                       static_cast<const float2 *>(spec), n,
                       n_cand, r, z, power, dp_dr, dp_dz, taps, n_steps, s_r, s_z);
    return hipGetLastError();
}

hipError_t launch_refine_backward(const void *spec, int64_t n, int32_t n_cand, const double *r, const double *z,
                                  const double *grad_p, double *grad_r, double *grad_z, int32_t taps, hipStream_t st) {
    if (n_cand == 0) return hipSuccess;
    const int per = taps <= 32 ? 2 : 1;   // candidates per wave
    hipLaunchKernelGGL(k_refine_backward, dim3((unsigned)((n_cand + per - 1) / per)), dim3(64), 0, st,
                       static_cast<const float2 *>(spec), n, n_cand, r, z, grad_p, grad_r, grad_z, taps);
    return hipGetLastError();
}

}  // namespace fdas
