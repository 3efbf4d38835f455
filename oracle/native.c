/*
 * Plain C loops for the oracle (test infrastructure only; the imaging library
 * never links this).  Built with gcc -O2 -fopenmp, no fast-math.
 *
 * oracle_grid_accumulate: the convolutional gridding sum of Eq. 3 with a
 *   separable kernel, one visibility at a time, into one complex float64 plane.
 * oracle_dft: the direct sum over visibilities that inverts Eq. 1 (with the
 *   w-term), evaluated at a list of pixels.
 * oracle_degrid: the transpose of oracle_grid_accumulate: each visibility reads
 *   the W x W cells its taps cover, weighted by the same separable kernel.
 * oracle_kb_eval: the Kaiser-Bessel kernel of the gridding step (Sec. 2, Jackson et al.
 *   1991) at a list of offsets, with I0 by its power series.
 */
#include <math.h>
#include <stdint.h>

/* I0(z) = sum_k (z^2/4)^k / (k!)^2: term_k = term_{k-1} * (z^2/4) / k^2, summed until a term
   is at most 1e-17 of the running sum (the same series and stopping rule as oracle/kb.py). */
static double i0_series(double z)
{
    const double q = 0.25 * z * z;
    double term = 1.0, total = 1.0;
    for (int k = 1; k <= 500; ++k) {
        term = term * q / ((double)k * (double)k);
        total = total + term;
        if (term <= 1e-17 * total) break;
    }
    return total;
}

/* out[i] = G(t[i]) = I0(beta sqrt(1 - (2 t / W)^2)) / I0(beta) for |t| <= W/2, else 0. */
void oracle_kb_eval(int64_t count, const double *t, int64_t support, double beta, double *out)
{
    const double norm = i0_series(beta);
    for (int64_t i = 0; i < count; ++i) {
        double s = 2.0 * t[i] / (double)support;
        double a = 1.0 - s * s;
        if (a < 0.0) a = 0.0;
        out[i] = fabs(t[i]) <= 0.5 * (double)support ? i0_series(beta * sqrt(a)) / norm : 0.0;
    }
}

/* grid[(p0+b)*n + q0+a] += wv * gx[a] * gy[b] for every visibility r in idx. */
void oracle_grid_accumulate(int64_t n, int64_t support, int64_t count,
                            const int64_t *idx, const int64_t *p0, const int64_t *q0,
                            const double *wv_re, const double *wv_im,
                            const double *gx, const double *gy, double *grid /* [n][n][2] */)
{
    for (int64_t c = 0; c < count; ++c) {
        int64_t r = idx[c];
        for (int64_t b = 0; b < support; ++b) {
            double gyb = gy[r * support + b];
            for (int64_t a = 0; a < support; ++a) {
                double g = gx[r * support + a] * gyb;
                int64_t cell = (p0[r] + b) * n + (q0[r] + a);
                grid[2 * cell] += wv_re[r] * g;
                grid[2 * cell + 1] += wv_im[r] * g;
            }
        }
    }
}

/*
 * out[p] = sum_m wv[m] * exp(+2 pi i (u[m] l[p] + v[m] mm[p] + w[m] nm1[p])) for each pixel p.
 * u, v, w in wavelengths; l, mm direction cosines; nm1 = n - 1.
 * The phase in cycles is reduced by its nearest integer before the 2 pi multiply.
 */
void oracle_dft(int64_t nvis, const double *u, const double *v, const double *w,
                const double *wv_re, const double *wv_im,
                int64_t npix, const double *l, const double *mm, const double *nm1,
                double *out /* [npix][2] */)
{
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
        double sr = 0.0, si = 0.0;
        for (int64_t m = 0; m < nvis; ++m) {
            double cyc = u[m] * l[p] + v[m] * mm[p] + w[m] * nm1[p];
            cyc -= nearbyint(cyc);
            double ph = two_pi * cyc;
            double c = cos(ph), s = sin(ph);
            sr += wv_re[m] * c - wv_im[m] * s;
            si += wv_re[m] * s + wv_im[m] * c;
        }
        out[2 * p] = sr;
        out[2 * p + 1] = si;
    }
}

/* out[c] = sum_{a,b} gx[c][a] * gy[c][b] * grid[p0[c]+b][q0[c]+a] for each of count rows. */
void oracle_degrid(int64_t n, int64_t support, int64_t count, const int64_t *p0, const int64_t *q0,
                   const double *gx, const double *gy, const double *grid /* [n][n][2] */,
                   double *out /* [count][2] */)
{
    for (int64_t c = 0; c < count; ++c) {
        double sr = 0.0, si = 0.0;
        for (int64_t b = 0; b < support; ++b) {
            double gyb = gy[c * support + b];
            for (int64_t a = 0; a < support; ++a) {
                double g = gx[c * support + a] * gyb;
                int64_t cell = (p0[c] + b) * n + (q0[c] + a);
                sr += grid[2 * cell] * g;
                si += grid[2 * cell + 1] * g;
            }
        }
        out[2 * c] = sr;
        out[2 * c + 1] = si;
    }
}
