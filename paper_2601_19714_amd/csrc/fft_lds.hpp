// Batched 1D complex FFTs of compile-time length held in LDS, for a whole work-group.
//
// Transform (the sign of Eq. 2, unnormalised):  X[j] = sum_q x[q] exp(+2 pi i q j / N),
// N = 2^LOG2N, applied to ROWS rows stored back to back (row r at element r*N, every
// element index passed through lds_pad).  Stockham autosort: each pass reads R inputs
// a stride N/R apart, twiddles them, runs an R-point DFT in registers and writes the R
// outputs a stride L apart, so the result ends in natural order with no bit reversal.
// Pass layout on a base radix R (8 here): radix R first, then one smaller-radix pass when
// LOG2N is not a multiple of log2 R, then radix R.  Twiddles come from a table
// tw[t] = exp(+2 pi i t / N) built in float64 on the host.  Every pass is written for NT
// threads with NT * R >= ROWS * N.
#pragma once

#include "device_common.hpp"

namespace wsimg {

template <typename C> __device__ __forceinline__ void dft2(C& a, C& b) {
    C t = a; a = cadd(t, b); b = csub(t, b);
}

template <typename C> __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
    C t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = cmuli(csub(a1, a3));
    a0 = cadd(t0, t2); a2 = csub(t0, t2); a1 = cadd(t1, t3); a3 = csub(t1, t3);
}

// a * exp(+2 pi i e / 16) for the exponents a 4 x 4 split needs
template <typename C> __device__ __forceinline__ C tw16(C a, int e) {
    using R = decltype(C::x);
    const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173, r2 = (R)0.70710678118654752440;
    switch (e) {
        case 0: return a;
        case 1: return cmul(a, cmake<C>(c1, s1));
        case 2: return cmake<C>(r2 * (a.x - a.y), r2 * (a.x + a.y));
        case 3: return cmul(a, cmake<C>(s1, c1));
        case 4: return cmuli(a);
        case 6: return cmake<C>(-r2 * (a.x + a.y), r2 * (a.x - a.y));
        case 9: return cmul(a, cmake<C>(-c1, -s1));
        default: return a;
    }
}

template <typename C> __device__ __forceinline__ void dft8(C* x) {
    // n = 2 n1 + n2, m = m1 + 4 m2
    dft4(x[0], x[2], x[4], x[6]);
    dft4(x[1], x[3], x[5], x[7]);
    x[3] = tw16(x[3], 2);     // m1 = 1: exp(2 pi i / 8)
    x[5] = tw16(x[5], 4);     // m1 = 2
    x[7] = tw16(x[7], 6);     // m1 = 3
    dft2(x[0], x[1]); dft2(x[2], x[3]); dft2(x[4], x[5]); dft2(x[6], x[7]);
    C y[8];
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) { y[m1] = x[2 * m1]; y[m1 + 4] = x[2 * m1 + 1]; }
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = y[i];
}

template <typename C> __device__ __forceinline__ void dft16(C* x) {
    // n = 4 n1 + n2, m = m1 + 4 m2
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(x[n2], x[n2 + 4], x[n2 + 8], x[n2 + 12]);
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int m1 = 1; m1 < 4; ++m1) x[n2 + 4 * m1] = tw16(x[n2 + 4 * m1], n2 * m1);
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) dft4(x[4 * m1], x[4 * m1 + 1], x[4 * m1 + 2], x[4 * m1 + 3]);
    C y[16];
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1)
#pragma unroll
        for (int m2 = 0; m2 < 4; ++m2) y[m1 + 4 * m2] = x[4 * m1 + m2];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = y[i];
}

template <int RAD, typename C> __device__ __forceinline__ void dft_small(C* x) {
    if constexpr (RAD == 2) dft2(x[0], x[1]);
    else if constexpr (RAD == 4) dft4(x[0], x[1], x[2], x[3]);
    else if constexpr (RAD == 8) dft8(x);
    else dft16(x);
}

// x[m] *= tw[(m k) << TWSHIFT] for m = 1 .. RAD-1.  With WSIMG_TW_DERIVE = 1 or 2 a
// radix-8 (radix-4) pass reads the powers m = 1, 2, 4 (1, 2) from the table and forms the
// others as their products (one extra rounding each), so fewer twiddles stay live in
// registers when a kernel keeps them across its loop; with 2 (the default) the products are
// formed at every use even where the compiler would hoist them (the stacking kernel then
// holds 111 instead of 128 + 48 spilled registers).
#ifndef WSIMG_TW_DERIVE
#define WSIMG_TW_DERIVE 2
#endif
template <typename C> __device__ __forceinline__ C opaque_val(C v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y));
    return v;
}

template <int RAD, int TWSHIFT, typename C>
__device__ __forceinline__ void twiddle_inputs(C* x, const C* __restrict__ tw, int k) {
    if constexpr (WSIMG_TW_DERIVE && RAD == 8) {
        C w1 = tw[k << TWSHIFT], w2 = tw[(2 * k) << TWSHIFT], w4 = tw[(4 * k) << TWSHIFT];
        if constexpr (WSIMG_TW_DERIVE == 2) { w1 = opaque_val(w1); w2 = opaque_val(w2); w4 = opaque_val(w4); }
        const C w3 = cmul(w1, w2);
        x[1] = cmul(x[1], w1);
        x[2] = cmul(x[2], w2);
        x[3] = cmul(x[3], w3);
        x[4] = cmul(x[4], w4);
        x[5] = cmul(x[5], cmul(w1, w4));
        x[6] = cmul(x[6], cmul(w2, w4));
        x[7] = cmul(x[7], cmul(w3, w4));
    } else if constexpr (WSIMG_TW_DERIVE && RAD == 4) {
        const C w1 = tw[k << TWSHIFT], w2 = tw[(2 * k) << TWSHIFT];
        x[1] = cmul(x[1], w1);
        x[2] = cmul(x[2], w2);
        x[3] = cmul(x[3], cmul(w1, w2));
    } else {
#pragma unroll
        for (int m = 1; m < RAD; ++m) x[m] = cmul(x[m], tw[(m * k) << TWSHIFT]);
    }
}

template <int V> struct Log2Of {
    static constexpr int value = V == 2 ? 1 : V == 4 ? 2 : V == 8 ? 3 : 4;          // radices
    static constexpr int value_any = V <= 1 ? 0 : 1 + Log2Of<(V > 1 ? V / 2 : 1)>::value_any;
};
template <> struct Log2Of<1> { static constexpr int value = 0; static constexpr int value_any = 0; };

// Pass layout of an N = 2^LOG2N transform on a base radix R = 2^LOGR (R elements per thread):
// [R (first)] [one radix-2^(LOG2N mod LOGR) pass when LOG2N is not a multiple of LOGR] [R ...].
template <int LOG2N, int LOGR> struct FftPlan {
    static constexpr int REM = LOG2N % LOGR;
    // radix (log2) of the last pass; the only pass when LOG2N <= LOGR
    static constexpr int LAST_LOG = LOG2N <= LOGR ? LOG2N : ((LOG2N < 2 * LOGR && REM) ? REM : LOGR);
    // log2 L at which the last pass starts
    static constexpr int LAST_L = LOG2N - LAST_LOG;
};

// One Stockham pass (LDS to LDS) at sub-length L = 2^LOG2L, for NT threads holding E elements
// each (E = 8 or 16; a radix-RAD pass gives each thread E / RAD butterflies).
template <int RAD, int LOG2N, int LOG2L, int ROWS, int NT, typename C>
__device__ __forceinline__ void stockham_pass(C* lds, const C* __restrict__ tw) {
    constexpr int LOGR = Log2Of<RAD>::value;
    constexpr int LSUB = LOG2N - LOGR;                     // log2(N / RAD)
    constexpr int NBF = ROWS << LSUB;
    constexpr int BPT = (NBF + NT - 1) / NT;               // butterflies per thread
    constexpr int L = 1 << LOG2L;
    constexpr int TWSHIFT = LOG2N - LOG2L - LOGR;
    const int tid = threadIdx.x;
    C x[BPT][RAD];
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
        const int g = tid + t * NT;
        if (NBF % NT == 0 || g < NBF) {
            const int r = g >> LSUB, b = g & ((1 << LSUB) - 1);
            const int base = (r << LOG2N) + b;
#pragma unroll
            for (int m = 0; m < RAD; ++m) x[t][m] = lds[lds_pad(base + (m << LSUB))];
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
        const int g = tid + t * NT;
        if (NBF % NT == 0 || g < NBF) {
            const int r = g >> LSUB, b = g & ((1 << LSUB) - 1);
            const int k = b & (L - 1), j = b >> LOG2L;
            if constexpr (L > 1) twiddle_inputs<RAD, TWSHIFT>(x[t], tw, k);
            dft_small<RAD>(x[t]);
            const int obase = (r << LOG2N) + (j << (LOG2L + LOGR)) + k;
#pragma unroll
            for (int m = 0; m < RAD; ++m) lds[lds_pad(obase + (m << LOG2L))] = x[t][m];
        }
    }
    __syncthreads();
}

// Passes from sub-length 2^LOG2L up to (not including) 2^STOP in the plan's layout: the
// odd-radix pass (if any) sits at LOG2L == LOGR, right after the first pass.
template <int LOG2N, int LOGR, int LOG2L, int STOP, int ROWS, int NT, typename C>
__device__ __forceinline__ void stockham_range(C* lds, const C* __restrict__ tw) {
    if constexpr (LOG2L < STOP) {
        constexpr int REM = LOG2N % LOGR;
        constexpr int LR = (REM != 0 && LOG2L == LOGR) ? REM : LOGR;
        stockham_pass<(1 << LR), LOG2N, LOG2L, ROWS, NT>(lds, tw);
        stockham_range<LOG2N, LOGR, LOG2L + LR, STOP, ROWS, NT>(lds, tw);
    }
}

// Full in-place transform of ROWS rows held in LDS (LOG2N > LOGR).
template <int LOG2N, int LOGR, int ROWS, int NT, typename C>
__device__ __forceinline__ void fft_rows_lds(C* lds, const C* __restrict__ tw) {
    static_assert(LOG2N > LOGR, "transforms start with a full-radix pass");
    stockham_pass<(1 << LOGR), LOG2N, 0, ROWS, NT>(lds, tw);
    stockham_range<LOG2N, LOGR, LOGR, LOG2N, ROWS, NT>(lds, tw);
}

// Last pass (L * RAD == N) from LDS into registers.  out[t * RAD + m] (E = 2^LOGR slots)
// holds output bin b + m * (N / RAD) of row (g >> LSUB), g = threadIdx.x + t * NT,
// b = g mod (N / RAD); slots of inactive threads are zero.  No barrier at the end.
template <int LOG2N, int LOGR, int ROWS, int NT, typename C>
__device__ __forceinline__ void fft_last_to_regs(const C* lds, const C* __restrict__ tw, C* out) {
    constexpr int LLOG = FftPlan<LOG2N, LOGR>::LAST_LOG;
    constexpr int RAD = 1 << LLOG;
    constexpr int LSUB = LOG2N - LLOG;
    constexpr int NBF = ROWS << LSUB;
    constexpr int BPT = (1 << LOGR) / RAD;
    const int tid = threadIdx.x;
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
        const int g = tid + t * NT;
        C x[RAD];
        if (g < NBF) {
            const int r = g >> LSUB, b = g & ((1 << LSUB) - 1);
            const int base = (r << LOG2N) + b;
#pragma unroll
            for (int m = 0; m < RAD; ++m) x[m] = lds[lds_pad(base + (m << LSUB))];
            twiddle_inputs<RAD, 0>(x, tw, b);
            dft_small<RAD>(x);
        } else {
#pragma unroll
            for (int m = 0; m < RAD; ++m) x[m] = cmake<C>(0, 0);
        }
#pragma unroll
        for (int m = 0; m < RAD; ++m) out[t * RAD + m] = x[m];
    }
}

// Row (image column of the block) c and bin i' held by register slot s of thread tid after
// fft_last_to_regs.
template <int LOG2N, int LOGR, int ROWS, int NT>
__device__ __forceinline__ bool last_slot(int tid, int s, int& c, int& ip) {
    constexpr int LLOG = FftPlan<LOG2N, LOGR>::LAST_LOG;
    constexpr int LSUB = LOG2N - LLOG;
    const int t = s >> LLOG, m = s & ((1 << LLOG) - 1);
    const int g = tid + t * NT;
    if (g >= (ROWS << LSUB)) return false;
    c = g >> LSUB;
    ip = (g & ((1 << LSUB) - 1)) + (m << LSUB);
    return true;
}

}  // namespace wsimg
