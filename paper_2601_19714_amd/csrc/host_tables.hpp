// Host-side constant tables of a plan, built in long double and rounded once to the
// plan's precision:
//   * per-tap Kaiser-Bessel polynomials in the sub-cell offset f in [-1/2, 1/2]
//     (Chebyshev interpolation of G(a - (W-1)/2 - f), converted to the monomial basis);
//   * the reciprocal grid-correction taper 1/C(xi) at xi = (i - n/2)/n;
//   * FFT twiddles exp(+2 pi i t / n).
// G(t) = I0(beta sqrt(1 - (2t/W)^2)) / I0(beta) is the Kaiser-Bessel kernel named in Sec. 2
// (Jackson et al. 1991); C is its continuous Fourier transform,
//   C(xi) = (W / I0(beta)) sinh(sqrt(beta^2 - (pi W xi)^2)) / sqrt(beta^2 - (pi W xi)^2).
#pragma once

#include <cmath>
#include <vector>

namespace wsimg {
namespace host {

using ld = long double;
static const ld kPiL = 3.141592653589793238462643383279502884L;

// I0 by its power series, summed until the term is below 1e-21 of the sum.
inline ld bessel_i0(ld z) {
    const ld q = 0.25L * z * z;
    ld term = 1.0L, sum = 1.0L;
    for (int k = 1; k < 1000; ++k) {
        term *= q / ((ld)k * (ld)k);
        sum += term;
        if (term < 1e-21L * sum) break;
    }
    return sum;
}

inline ld kb_kernel(ld t, int W, ld beta) {
    const ld s = 2.0L * t / (ld)W;
    if (std::fabs(t) > 0.5L * (ld)W) return 0.0L;
    ld a = 1.0L - s * s;
    if (a < 0.0L) a = 0.0L;
    return bessel_i0(beta * std::sqrt(a)) / bessel_i0(beta);
}

inline ld kb_transform(ld xi, int W, ld beta) {
    const ld a2 = beta * beta - (kPiL * (ld)W * xi) * (kPiL * (ld)W * xi);
    ld shape;
    if (a2 > 0.0L) { const ld r = std::sqrt(a2); shape = std::sinh(r) / r; }
    else if (a2 < 0.0L) { const ld r = std::sqrt(-a2); shape = std::sin(r) / r; }
    else shape = 1.0L;
    return (ld)W / bessel_i0(beta) * shape;
}

// coef[a * (deg + 1) + d]: G(a - half - f) ~= sum_d coef[a][d] f^d on f in [-1/2, 1/2].
inline std::vector<ld> kb_tap_polynomials(int W, ld beta, int deg) {
    const int half = (W - 1) / 2, np = deg + 1;
    std::vector<ld> out((size_t)W * np, 0.0L);
    std::vector<ld> g(np), cheb(np), mono(np), tprev(np), tcur(np), tnext(np);
    for (int a = 0; a < W; ++a) {
        for (int k = 0; k < np; ++k) {
            const ld x = std::cos(kPiL * ((ld)k + 0.5L) / (ld)np);   // node in [-1, 1], f = x/2
            g[k] = kb_kernel((ld)(a - half) - 0.5L * x, W, beta);
        }
        for (int j = 0; j < np; ++j) {
            ld s = 0.0L;
            for (int k = 0; k < np; ++k) s += g[k] * std::cos(kPiL * (ld)j * ((ld)k + 0.5L) / (ld)np);
            cheb[j] = (j == 0 ? 1.0L : 2.0L) * s / (ld)np;
        }
        // sum_j cheb[j] T_j(x) as monomials in x, by T_{j+1} = 2x T_j - T_{j-1}
        std::fill(mono.begin(), mono.end(), 0.0L);
        std::fill(tprev.begin(), tprev.end(), 0.0L);
        std::fill(tcur.begin(), tcur.end(), 0.0L);
        tprev[0] = 1.0L;                  // T_0
        if (np > 1) tcur[1] = 1.0L;       // T_1
        mono[0] += cheb[0];
        if (np > 1) for (int d = 0; d < np; ++d) mono[d] += cheb[1] * tcur[d];
        for (int j = 2; j < np; ++j) {
            for (int d = 0; d < np; ++d)
                tnext[d] = (d > 0 ? 2.0L * tcur[d - 1] : 0.0L) - tprev[d];
            for (int d = 0; d < np; ++d) mono[d] += cheb[j] * tnext[d];
            tprev = tcur;
            tcur = tnext;
        }
        // x = 2 f
        ld p2 = 1.0L;
        for (int d = 0; d < np; ++d) { out[(size_t)a * np + d] = mono[d] * p2; p2 *= 2.0L; }
    }
    return out;
}

// 1 / C(xi) for image pixels i = 0 .. n-1, xi = (i - n/2) / n_grid (n_grid = n, or 2n for a
// padded grid).
inline std::vector<ld> inverse_taper(int n, int n_grid, int W, ld beta) {
    std::vector<ld> out(n);
    for (int i = 0; i < n; ++i) out[i] = 1.0L / kb_transform((ld)(i - n / 2) / (ld)n_grid, W, beta);
    return out;
}

inline void twiddles(int n, std::vector<ld>& re, std::vector<ld>& im) {
    re.resize(n); im.resize(n);
    for (int t = 0; t < n; ++t) {
        const ld a = 2.0L * kPiL * (ld)t / (ld)n;
        re[t] = std::cos(a);
        im[t] = std::sin(a);
    }
}

}  // namespace host
}  // namespace wsimg
