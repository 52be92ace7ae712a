/* Direct (no-FFT) f-fdot plane, double precision -- TEST INFRASTRUCTURE ONLY.
 *
 * The plane is the correlation of the normalised spectrum with every
 * acceleration template (Section "Detailed explanation": the signal is
 * convolved with all templates, giving the f-fdot plane; a pulsar shows as a
 * peak).  The paper computes it through the convolution theorem with
 * overlap-save; the plain definition computed here is
 *
 *     P[j, r] = | sum_{m=-M/2}^{M/2-1} X[r - m] * g_j[m] |^2 ,  X = 0 outside [0, N)
 *
 * (8M + 3 flops per cell).  No blocking, no FFT, OpenMP over r only.
 * Complex arrays are interleaved (re, im) doubles; g is n_z x M, column i is
 * tap m = i - M/2.
 */
#include <stdint.h>
#include <omp.h>

int fdas_oracle_threads(void) { return omp_get_max_threads(); }

static void cell(const double *x, int64_t n, const double *g, int32_t m_taps,
                 int64_t r, double *out_re, double *out_im)
{
    double re = 0.0, im = 0.0;
    const int32_t half = m_taps / 2;
    for (int32_t i = 0; i < m_taps; ++i) {
        const int64_t k = r - (int64_t)(i - half);
        if (k < 0 || k >= n) continue;
        const double xr = x[2 * k], xi = x[2 * k + 1];
        const double gr = g[2 * i], gi = g[2 * i + 1];
        re += xr * gr - xi * gi;
        im += xr * gi + xi * gr;
    }
    *out_re = re;
    *out_im = im;
}

/* Plane rows 0..n_z-1 for columns r in [r0, r1); out is n_z x (r1 - r0). */
void fdas_oracle_plane(const double *x, int64_t n, const double *g, int32_t n_z,
                       int32_t m_taps, int64_t r0, int64_t r1, double *out)
{
    const int64_t w = r1 - r0;
#pragma omp parallel for schedule(static)
    for (int64_t r = r0; r < r1; ++r) {
        for (int32_t j = 0; j < n_z; ++j) {
            double re, im;
            cell(x, n, g + 2 * (int64_t)j * m_taps, m_taps, r, &re, &im);
            out[(int64_t)j * w + (r - r0)] = re * re + im * im;
        }
    }
}

/* Individual cells (j[i], r[i]) -> out[i]; also returns the complex sum. */
void fdas_oracle_cells(const double *x, int64_t n, const double *g, int32_t m_taps,
                       const int32_t *j, const int64_t *r, int64_t count,
                       double *power, double *amp)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        double re, im;
        cell(x, n, g + 2 * (int64_t)j[i] * m_taps, m_taps, r[i], &re, &im);
        power[i] = re * re + im * im;
        if (amp) { amp[2 * i] = re; amp[2 * i + 1] = im; }
    }
}
