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
// composite 16-point Gauss-Legendre quadrature with panels of at most two
// turns of phase (the rule's error bound for e^{i phi} over 4 pi of phase is
// below 1e-17; against panels four times finer the moments agree to
// 1.1e-15 for |q| <= 17.5, |z| <= 0.05).  The closed form divides by z
// twice: its numerators are O(z) with absolute errors near
// eps (1 + 2 pi |q| |A|), so M2 carries about eps 2 pi |q| / (2 pi z)^2,
// 2e-12 at z = 0.05 and |q| = 16 taps out -- far inside the refinement's
// bars -- while the quadrature costs about 8 (|q| + |z|) + 16 evaluations
// of exp(i phi) per tap, so the few candidates near z = 0 still take
// longest.
//
// Ascent step (the paper prints none): a Newton step on the analytic
// curvature of an isolated peak, r += s_r 3 / (2 pi^2 P) dP/dr and
// z += s_z 90 / (pi^2 P) dP/dz.
//
// One wave per candidate.  Up to 32 taps, lanes 2 t and 2 t + 1 share tap t:
// each evaluates one of the two end points of its closed form (or every
// other panel of its quadrature) and the pair swaps the results, so a lane
// runs one series or continued fraction per evaluation and the wave twice as
// many candidates' worth of them are in flight; with more taps lane t holds
// tap t.  The three sums are reduced by an XOR butterfly over the wave
// (fixed order, the same on every lane; the second lane of a pair adds
// zeros), so every lane sees the same (r, z) trajectory.
// Everything is FP64: a bin index near 4e6 has an FP32 spacing of half a
// bin.
#include "internal.hpp"
#include "response.hpp"

namespace fdas {

constexpr double kClosedFormZ = 0.05;

// Panels of the quadrature of A and its moments: at most two turns of the
// phase pi (2 q u + z u^2), |phase'| <= pi (2 |q| + 2 |z|) on [0, 1].
__device__ __forceinline__ int quad_panels(double q, double z) {
    return (int)ceil(0.5 * (fabs(q) + fabs(z))) + 1;
}

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
    const int npan = quad_panels(q, z);
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

// One end point y of the closed form for z > 0: G(|y|) and E(|y|) from one
// series (|y| < 2) or continued fraction, the values aux_g and fresnel_e
// form from it.
struct EndPoint {
    cd g, e;
};
__device__ inline EndPoint end_point(double ay) {
    EndPoint p;
    if (ay < 2.0) {
        p.e = fresnel_series(ay);
        p.g = (mk(0.5, 0.5) - p.e) * conj(expipi(0.5 * ay * ay));
    } else {
        p.g = aux_g(ay);
        p.e = mk(0.5, 0.5) - p.g * expipi(0.5 * ay * ay);
    }
    return p;
}

__device__ __forceinline__ cd swap_pair(cd v) { return {__shfl_xor(v.re, 1, 64), __shfl_xor(v.im, 1, 64)}; }

// A(q, z) for z > 0 by the lane pair (lanes 2 t + e, e = 0, 1; both call it):
// lane e evaluates end point Y1 (e = 0) or Y2, then both combine them as
// response_pos does.
__device__ cd response_pos_pair(double q, double z, int e) {
    const double s = sqrt(2.0 / z);
    const double y1 = q * s, y2 = (q + z) * s;
    const double rt = sqrt(2.0 * z);
    const EndPoint own = end_point(fabs(e ? y2 : y1));
    const EndPoint other = {swap_pair(own.g), swap_pair(own.e)};
    const EndPoint p1 = e ? other : own, p2 = e ? own : other;
    if (y1 >= 0.0) {
        cd v = p1.g - p2.g * expipi(2.0 * q + z);
        return (1.0 / rt) * v;
    }
    if (y2 <= 0.0) {
        cd v = p2.g * expipi(2.0 * q + z) - p1.g;
        return (1.0 / rt) * v;
    }
    cd d = p2.e - mk(-p1.e.re, -p1.e.im);   // E(Y2) - E(Y1), Y1 < 0 < Y2
    return (1.0 / rt) * (conj(expipi(q * q / z)) * d);
}

// response_d by the lane pair of one tap.
__device__ void response_d_pair(double q, double z, int e, cd &A, cd &Aq, cd &Az) {
    const double twopi = 2.0 * M_PI;
    if (fabs(z) >= kClosedFormZ) {
        A = z > 0.0 ? response_pos_pair(q, z, e) : conj(response_pos_pair(-q, -z, e));
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
    // the quadrature: lane e takes panels e, e + 2, ...; the pair adds halves
    const int npan = quad_panels(q, z);
    cd m0 = {0, 0}, m1 = {0, 0}, m2 = {0, 0};
    for (int pn = e; pn < npan; pn += 2) {
        for (int i = 0; i < 16; ++i) {
            const double u = (pn + kGLx[i]) / npan;
            const double wt = kGLw[i] / npan;
            const cd ex = expipi(2.0 * q * u + z * u * u);
            m0 = m0 + wt * ex;
            m1 = m1 + (wt * u) * ex;
            m2 = m2 + (wt * u * u) * ex;
        }
    }
    m0 = m0 + swap_pair(m0);
    m1 = m1 + swap_pair(m1);
    m2 = m2 + swap_pair(m2);
    A = m0;
    Aq = {-twopi * m1.im, twopi * m1.re};
    Az = {-M_PI * m2.im, M_PI * m2.re};
}

// Sum over the 64 lanes of the wave.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct RefineOut {
    double P, dPr, dPz;
};

// Every lane of the wave returns the same values.
__device__ RefineOut eval_point(const float2 *spec, int64_t n, double r, double z, int taps, int lane) {
    const bool paired = taps <= 32;
    const int tap = paired ? lane >> 1 : lane;
    const int e = paired ? lane & 1 : 0;
    cd F = {0, 0}, Fr = {0, 0}, Fz = {0, 0};
    if (tap < taps) {
        const int64_t k = (int64_t)floor(r) - taps / 2 + 1 + tap;
        if (k >= 0 && k < n) {   // the same for both lanes of a pair
            const float2 xv = spec[k];
            const cd x = {(double)xv.x, (double)xv.y};
            cd A, Aq, Az;
            if (paired)
                response_d_pair(r - 0.5 * z - (double)k, z, e, A, Aq, Az);
            else
                response_d(r - 0.5 * z - (double)k, z, A, Aq, Az);
            if (e == 0) {
                F = x * conj(A);
                Fr = x * conj(Aq);
                Fz = x * conj(Az - 0.5 * Aq);
            }
        }
    }
    F = {wave_sum(F.re), wave_sum(F.im)};
    Fr = {wave_sum(Fr.re), wave_sum(Fr.im)};
    Fz = {wave_sum(Fz.re), wave_sum(Fz.im)};
    RefineOut o;
    o.P = F.re * F.re + F.im * F.im;
    o.dPr = 2.0 * (F.re * Fr.re + F.im * Fr.im);
    o.dPz = 2.0 * (F.re * Fz.re + F.im * Fz.im);
    return o;
}

__global__ void __launch_bounds__(64) k_refine(const float2 *spec, int64_t n, int32_t n_cand, double *r, double *z,
                                               double *power, double *dp_dr, double *dp_dz, int32_t taps,
                                               int32_t n_steps, double s_r, double s_z) {
    const int cand = blockIdx.x;
    if (cand >= n_cand) return;   // the whole wave
    const int lane = (int)threadIdx.x;
    double rr = r[cand], zz = z[cand];
    const double pi2 = M_PI * M_PI;
    for (int it = 0; it < n_steps; ++it) {
        const RefineOut o = eval_point(spec, n, rr, zz, taps, lane);
        const double Ps = fmax(o.P, 1e-30);
        rr += s_r * 3.0 / (2.0 * pi2 * Ps) * o.dPr;
        zz += s_z * 90.0 / (pi2 * Ps) * o.dPz;
    }
    const RefineOut o = eval_point(spec, n, rr, zz, taps, lane);
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
    const int cand = blockIdx.x;
    if (cand >= n_cand) return;
    const int lane = (int)threadIdx.x;
    const RefineOut o = eval_point(spec, n, r[cand], z[cand], taps, lane);
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
    hipLaunchKernelGGL(k_refine, dim3((unsigned)n_cand), dim3(64), 0, st,
                       static_cast<const float2 *>(spec), n,
                       n_cand, r, z, power, dp_dr, dp_dz, taps, n_steps, s_r, s_z);
    return hipGetLastError();
}

hipError_t launch_refine_backward(const void *spec, int64_t n, int32_t n_cand, const double *r, const double *z,
                                  const double *grad_p, double *grad_r, double *grad_z, int32_t taps, hipStream_t st) {
    if (n_cand == 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine_backward, dim3((unsigned)n_cand), dim3(64), 0, st,
                       static_cast<const float2 *>(spec), n, n_cand, r, z, grad_p, grad_r, grad_z, taps);
    return hipGetLastError();
}

}  // namespace fdas
