// Device-side helpers shared by the imaging kernels: complex arithmetic on HIP
// vector types, the per-row geometry of the gridding step, and the LDS index padding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsimg {

constexpr double kCLight = 299792458.0;   // m/s
constexpr int kMaxSupport = 15;           // largest odd Kaiser-Bessel support
constexpr int kInvalidKey = -1;

template <typename R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

template <typename C> __device__ __forceinline__ C cmake(decltype(C::x) re, decltype(C::x) im) {
    C r; r.x = re; r.y = im; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by +i
template <typename C> __device__ __forceinline__ C cmuli(C a) { return cmake<C>(-a.y, a.x); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cmake<C>(a.x * s, a.y * s); }

// LDS element index with one pad slot per 2^WSIMG_LDS_PAD_SHIFT elements: keeps the strided
// Stockham writes and the butterfly reads off common banks (one per 32: a 4096^2 image 2.87 ->
// 2.85 ms and an 8192^2 one 48.4 -> 47.7 ms against one per 16; one per 8 was slower).
#ifndef WSIMG_LDS_PAD_SHIFT
#define WSIMG_LDS_PAD_SHIFT 5
#endif
__device__ __forceinline__ int lds_pad(int e) { return e + (e >> WSIMG_LDS_PAD_SHIFT); }
// Hide a (wave-uniform) pointer's value from the optimiser.  Used on the twiddle table at
// the top of loops over strips or planes, so its loads stay inside each FFT pass instead of
// being hoisted out of the loop into registers the passes need.
template <typename T>
__device__ __forceinline__ const T* opaque_ptr(const T* p) {
    asm volatile("" : "+s"(p));
    return p;
}

__host__ __device__ __forceinline__ int lds_padded_elems(int e) { return e + (e >> WSIMG_LDS_PAD_SHIFT) + 1; }
// padded element count rounded up to an even number, so a double array can follow it
constexpr int lds_padded_elems_c(int e) { return (e + (e >> WSIMG_LDS_PAD_SHIFT) + 2) & ~1; }

// Grid position of one row, computed in float64 with the operation order the imaging
// definition uses:  u = (uvw_u * freq) / c,  x = u / du + n/2  (same for v, y; w likewise
// without the offset).  No contraction into FMAs, so every rounding is the plain IEEE one.
struct RowGeom {
    double x, y, w;
    double cx, cy;    // floor(x + 1/2), floor(y + 1/2): the cell nearest to the row
    bool keep;        // finite uvw and weight, all taps on the grid
    bool flip;        // w-folding replaced the row by its conjugate partner
};

// fold: w-folding, a row with w < 0 becomes (-u, -v, -w) (its visibility is conjugated by the
// caller): V(-u, -v, -w) = conj V(u, v, w) for a real sky, and the planes span |w| only.
__device__ __forceinline__ RowGeom row_geometry(const double* __restrict__ uvw, int64_t m, double freq,
                                                double du, double half_n, double wt, int n, int support,
                                                bool fold) {
#pragma clang fp contract(off)
    RowGeom g;
    double uu = uvw[3 * m + 0], vv = uvw[3 * m + 1], ww = uvw[3 * m + 2];
    g.flip = fold && ww < 0.0;
    if (g.flip) { uu = -uu; vv = -vv; ww = -ww; }
    const double u = uu * freq / kCLight;
    const double v = vv * freq / kCLight;
    g.w = ww * freq / kCLight;
    g.x = u / du + half_n;
    g.y = v / du + half_n;
    g.cx = floor(g.x + 0.5);
    g.cy = floor(g.y + 0.5);
    const double h = (double)((support - 1) / 2);
    const double fq = g.cx - h, fp = g.cy - h;
    const double last = (double)(n - 1), span = (double)(support - 1);
    const bool finite = isfinite(uu) && isfinite(vv) && isfinite(ww) && isfinite(wt);
    g.keep = finite && (fq >= 0.0) && (fq + span <= last) && (fp >= 0.0) && (fp + span <= last);
    return g;
}

// Plane index of a kept row: clamp(floor((w - w_lo) / dw), 0, nw - 1); 0 when dw == 0.
__device__ __forceinline__ int plane_index(double w, double w_lo, double dw, int nw) {
#pragma clang fp contract(off)
    if (dw == 0.0) return 0;
    double kf = floor((w - w_lo) / dw);
    if (!(kf >= 0.0)) return 0;
    if (kf > (double)(nw - 1)) return nw - 1;
    return (int)kf;
}

// The w-kernel across planes (support Ww = 2h + 1): a kept row's plane coordinate
// z = (w - w_lo) / dw + h, clamped to [h, nw - 1 - h] (h when dw = 0), its first w-tap plane
// k0 = floor(z + 1/2) - h and its offset f = z - (k0 + h) in [-1/2, 1/2): the row adds to
// planes k0 .. k0 + Ww - 1 with weights G_w(k - z) = tap (k - k0) of the w-kernel at f.
struct WTap {
    int k0;
    double f;
};
__device__ __forceinline__ WTap w_taps(double w, double w_lo, double dw, int nw, int h) {
#pragma clang fp contract(off)
    double z = (dw == 0.0) ? (double)h : (w - w_lo) / dw + (double)h;
    const double zlo = (double)h, zhi = (double)(nw - 1 - h);
    if (!(z >= zlo)) z = zlo;
    if (z > zhi) z = zhi;
    const double c = floor(z + 0.5);
    WTap t;
    t.k0 = (int)c - h;
    t.f = z - c;
    return t;
}

// C(xi) = (W / I0(beta)) sinh(r) / r with r = sqrt(beta^2 - (pi W xi)^2) (sin(r) / r when
// pi W |xi| > beta): the continuous Fourier transform of the Kaiser-Bessel kernel; scale is
// W / I0(beta).  Float64.
__device__ __forceinline__ double kb_transform(double xi, int W, double beta, double scale) {
    const double pw = 3.14159265358979323846 * (double)W * xi;
    const double a2 = beta * beta - pw * pw;
    const double r = sqrt(fabs(a2));
    double s;
    if (r < 1e-4) s = 1.0 + (a2 > 0.0 ? 1.0 : -1.0) * (r * r / 6.0);
    else if (a2 > 0.0) s = sinh(r) / r;
    else s = sin(r) / r;
    return scale * s;
}

// sin(2 pi t) and cos(2 pi t) for |t| <= 1/2 (t in turns), float64.  Quadrant reduction
// q = rint(4t), r = t - q/4 (exact), |r| <= 1/8; then the Taylor series of sin and cos of
// 2 pi r to degree 21 / 22 (truncation below 5e-16) and the quadrant rotation.
__device__ __forceinline__ void sincos_turn(double t, double* s, double* c) {
    const double q = rint(4.0 * t);
    const double r = t - 0.25 * q;
    const double r2 = r * r;
    double ps = 0.00113092374825179618777;
    ps = ps * r2 + -0.0120315859421206272332;
    ps = ps * r2 + 0.104229162208139841173;
    ps = ps * r2 + -0.718122301778500512232;
    ps = ps * r2 + 3.81995258484828212773;
    ps = ps * r2 + -15.0946425768229903918;
    ps = ps * r2 + 42.058693944897653145;
    ps = ps * r2 + -76.7058597530613858416;
    ps = ps * r2 + 81.6052492760750542034;
    ps = ps * r2 + -41.341702240399760234;
    ps = ps * r2 + 6.28318530717958647693;
    const double sr = ps * r;
    double pc = -0.000322991067207097788863;
    pc = pc * r2 + 0.00377983420068003937922;
    pc = pc * r2 + -0.0363828411425456707718;
    pc = pc * r2 + 0.28200596845579121507;
    pc = pc * r2 + -1.71439071108867206542;
    pc = pc * r2 + 7.90353637131846880421;
    pc = pc * r2 + -26.4262567833743974529;
    pc = pc * r2 + 60.2446413718766603627;
    pc = pc * r2 + -85.456817206693727736;
    pc = pc * r2 + 64.939394022668291491;
    pc = pc * r2 + -19.7392088021787172377;
    const double cr = pc * r2 + 1.0;
    const int qi = ((int)q) & 3;
    const double ss = (qi & 1) ? cr : sr, cc = (qi & 1) ? sr : cr;
    *s = (qi & 2) ? -ss : ss;
    *c = ((qi + 1) & 2) ? -cc : cc;
}

}  // namespace wsimg
