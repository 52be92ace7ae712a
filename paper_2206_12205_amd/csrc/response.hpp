// Double-precision acceleration response on the device.
//
// A(q, z) = int_0^1 exp(i pi (2 q u + z u^2)) du is the normalised Fourier
// response of a linearly drifting sinusoid (the method of Ransom et al. 2002,
// cited in Section "Introduction"; the paper gives no formula).  Completing
// the square expresses it through the Fresnel integral E(x) = C(x) + i S(x) =
// int_0^x exp(i pi t^2 / 2) dt:
//
//   z > 0:  A = exp(-i pi q^2 / z) / sqrt(2 z) * (E(Y2) - E(Y1)),
//           Y1 = q sqrt(2/z),  Y2 = (q + z) sqrt(2/z).
//
// With G(x) = (1 + i)/2 * erfcx(sqrt(pi)/2 (1 - i) x) for x >= 0 one has
// E(x) = (1 + i)/2 - G(x) exp(i pi x^2 / 2), which lets the large phases
// cancel analytically when Y1, Y2 share a sign:
//
//   Y1 >= 0:  A = (G(Y1) - G(Y2) exp(i pi (2q + z))) / sqrt(2 z)
//   Y2 <= 0:  A = (G(-Y2) exp(i pi (2q + z)) - G(-Y1)) / sqrt(2 z)
//
// z < 0 uses A(q, z) = conj(A(-q, -z)); z = 0 is Fourier interpolation
// exp(i pi q) sin(pi q) / (pi q); 0 < |z| < 1e-6 adds the first-order term
// z * dA/dz(q, 0) = z * i pi int_0^1 u^2 exp(2 pi i q u) du.
//
// Numerical methods (written for this library):
//   E(x), |x| < 2   Maclaurin series  sum_n (i pi/2)^n x^(2n+1) / (n! (2n+1))
//   erfcx(w)        Laplace continued fraction (Abramowitz & Stegun 7.1.14)
//                   evaluated bottom-up with 64 levels, used for |x| >= 2
//                   (relative error ~1e-15 there).
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

struct cd {
    double re, im;
};
__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cd conj(cd a) { return {a.re, -a.im}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    // Smith's algorithm, one reciprocal of the common denominator
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, inv = 1.0 / (b.re + r * b.im);
        return {(a.re + a.im * r) * inv, (a.im - a.re * r) * inv};
    }
    const double r = b.re / b.im, inv = 1.0 / (b.im + r * b.re);
    return {(a.re * r + a.im) * inv, (a.im * r - a.re) * inv};
}
// exp(i pi t) with t reduced mod 2 first
__device__ __forceinline__ cd expipi(double t) {
    // t mod 2 with the sign of t (fmod's value): t / 2, its truncation, twice
    // that and the difference are all exact in double precision
    const double tr = t - 2.0 * trunc(0.5 * t);
    double s, c;
    sincospi(tr, &s, &c);
    return {c, s};
}

constexpr double kSqrtPi = 1.7724538509055160273;

// Fresnel integral E(x) = C(x) + i S(x) for |x| < 2 by its Maclaurin series.
__device__ inline cd fresnel_series(double x) {
    const double a = 0.5 * M_PI * x * x;      // term ratio (i a) / (n + 1)
    cd term = {x, 0.0};                        // (i a)^n x / n!
    cd sum = {0.0, 0.0};
    // unrolled: 1 / (2 n + 1) and 1 / (n + 1) are constants, no division
#pragma unroll
    for (int n = 0; n < 48; ++n) {
        const double inv = 1.0 / (2 * n + 1);
        sum = sum + inv * term;
        // term *= i a / (n + 1)
        const double f = a * (1.0 / (n + 1));
        term = {-term.im * f, term.re * f};
    }
    return sum;
}

// erfcx(w) = exp(w^2) erfc(w), Re w > 0, by the Laplace continued fraction
// truncated after `depth` terms (evaluated from the tail).
__device__ inline cd erfcx_cf(cd w, int depth) {
    cd f = w;
    for (int k = depth; k >= 1; --k) f = w + cdiv(mk(0.5 * k, 0.0), f);
    return cdiv(mk(1.0 / kSqrtPi, 0.0), f);
}

// G(x) = (1 + i)/2 erfcx(sqrt(pi)/2 (1 - i) x), x >= 0 (so that
// E(x) = (1 + i)/2 - G(x) exp(i pi x^2 / 2)).  On that ray the fraction
// meets double precision (against a 400-term tail, in double) after 58 terms
// at x = 2, 27 at x = 3, 13 at x = 5 and 8 at x = 10; 12 + 220 / x^2 terms
// keep at least five to spare at every x >= 2.
__device__ inline cd aux_g(double x) {
    if (x >= 2.0) {
        const double s = 0.5 * kSqrtPi * x;
        return mk(0.5, 0.5) * erfcx_cf(mk(s, -s), 12 + (int)(220.0 / (x * x)));
    }
    // small x: from the series, no cancellation at this size
    cd e = fresnel_series(x);
    cd d = mk(0.5, 0.5) - e;
    return d * conj(expipi(0.5 * x * x));
}

// E(x) for any real x (odd function).
__device__ inline cd fresnel_e(double x) {
    const double ax = fabs(x);
    cd e;
    if (ax < 2.0) {
        e = fresnel_series(ax);
    } else {
        e = mk(0.5, 0.5) - aux_g(ax) * expipi(0.5 * ax * ax);
    }
    return x < 0.0 ? mk(-e.re, -e.im) : e;
}

// Response for z > 0.
__device__ inline cd response_pos(double q, double z) {
    const double s = sqrt(2.0 / z);
    const double y1 = q * s, y2 = (q + z) * s;
    const double rt = sqrt(2.0 * z);
    if (y1 >= 0.0) {
        cd v = aux_g(y1) - aux_g(y2) * expipi(2.0 * q + z);
        return (1.0 / rt) * v;
    }
    if (y2 <= 0.0) {
        cd v = aux_g(-y2) * expipi(2.0 * q + z) - aux_g(-y1);
        return (1.0 / rt) * v;
    }
    cd d = fresnel_e(y2) - fresnel_e(y1);
    return (1.0 / rt) * (conj(expipi(q * q / z)) * d);
}

// int_0^1 u^2 exp(a u) du for a = 2 pi i q.
__device__ inline cd moment2(double q) {
    const double w = 2.0 * M_PI * q;     // a = i w
    if (fabs(w) < 0.5) {
        // sum_n a^n / (n! (n + 3))
        cd term = {1.0, 0.0}, sum = {0.0, 0.0};
        for (int n = 0; n < 24; ++n) {
            sum = sum + (1.0 / (n + 3)) * term;
            term = mk(-term.im * w / (n + 1), term.re * w / (n + 1));
        }
        return sum;
    }
    // e^a (1/a - 2/a^2 + 2/a^3) - 2/a^3 with a = i w
    const cd a = {0.0, w};
    const cd ia = cdiv(mk(1.0, 0.0), a);
    const cd ia2 = ia * ia, ia3 = ia2 * ia;
    const cd ea = expipi(2.0 * q);
    return ea * (ia - 2.0 * ia2 + 2.0 * ia3) - 2.0 * ia3;
}

// 16-point Gauss-Legendre nodes and weights on [0, 1].
__device__ constexpr double kGLx[16] = {
    0.0052995325041750307, 0.0277124884633837,  0.067184398806084122, 0.1222977958224985,
    0.19106187779867811,   0.27099161117138632, 0.35919822461037054,  0.45249374508118129,
    0.54750625491881877,   0.64080177538962946, 0.72900838882861363,  0.80893812220132189,
    0.87770220417750155,   0.93281560119391593, 0.9722875115366163,   0.99470046749582497};
__device__ constexpr double kGLw[16] = {
    0.013576229705877019, 0.031126761969323853, 0.047579255841246296, 0.062314485627767015,
    0.074797994408288382, 0.08457825969750131,  0.091301707522461806, 0.094725305227534293,
    0.094725305227534293, 0.091301707522461806, 0.08457825969750131,  0.074797994408288382,
    0.062314485627767015, 0.047579255841246296, 0.031126761969323853, 0.013576229705877019};

// Response with a jerk term, A(q, z, w) = int_0^1 exp(i pi (2 q u + z u^2 +
// w u^3 / 3)) du: a sinusoid whose frequency (bins) runs r0 + z u + w u^2 / 2
// over the observation (w the change of the drift; w = 0 is A(q, z)).  No
// closed form: composite 16-point Gauss-Legendre quadrature with panels of
// at most two turns of phase (|phase'| <= pi (2|q| + 2|z| + |w|) on [0, 1];
// the rule's error bound over 4 pi of phase is below 1e-17, and against
// half-turn panels four times finer the sums agree to 3.8e-15 for |q| <= 140,
// |z| <= 120, |w| <= 100).
// Panels first, first + stride, ... of that quadrature (a part of the sum,
// so that a wave can split the panels over its lanes).
__device__ inline cd response_jerk_panels(double q, double z, double w, int first, int stride) {
    const int npan = (int)ceil(0.25 * (2.0 * fabs(q) + 2.0 * fabs(z) + fabs(w))) + 1;
    cd s = {0.0, 0.0};
    for (int pn = first; pn < npan; pn += stride) {
        for (int i = 0; i < 16; ++i) {
            const double u = (pn + kGLx[i]) / npan;
            const double wt = kGLw[i] / npan;
            s = s + wt * expipi(2.0 * q * u + z * u * u + w * u * u * u / 3.0);
        }
    }
    return s;
}

__device__ inline cd response_jerk(double q, double z, double w) { return response_jerk_panels(q, z, w, 0, 1); }

// A(q, z) for any real q, z.
__device__ inline cd response(double q, double z) {
    if (fabs(z) < 1e-6) {
        cd a0;
        if (q == 0.0) {
            a0 = {1.0, 0.0};
        } else {
            const double sn = sinpi(q) / (M_PI * q);
            a0 = sn * expipi(q);
        }
        if (z == 0.0) return a0;
        cd d = moment2(q);                       // dA/dz = i pi * moment2
        return a0 + z * (mk(0.0, M_PI) * d);
    }
    if (z > 0.0) return response_pos(q, z);
    return conj(response_pos(-q, -z));
}

}  // namespace fdas
