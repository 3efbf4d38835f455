// C ABI of the w-stacking imager: plan set-up, argument checks, launches.
// The declarations and their contracts are in include/wsimg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/wsimg.h"
#include "host_tables.hpp"
#include "kernels.hpp"

using namespace wsimg;

namespace {

thread_local std::string g_last_error;

wsimg_status fail(wsimg_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define WS_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? WSIMG_E_NOMEM : WSIMG_E_HIP,           \
                        std::string(#call) + ": " + hipGetErrorString(e_));                \
    } while (0)

const char* kStageNames[WSIMG_N_KERNELS] = {"zero_counts", "reduce", "key", "scan",
                                            "scatter", "origin_sort", "grid_rows", "cols_stack"};

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }

}  // namespace

struct wsimg_plan {
    wsimg_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t max_vis = 0;          // rows per call, all channels together
    int max_channels = 1;
    Geom g{};
    int nt1 = 0, nt2 = 0, nt2a = 0;  // threads of the gridding, stacking and prediction column work-groups
    int bs = 1;                      // image columns per stacking work-group
    int ba = 1;                      // image columns per prediction column work-group
    size_t lds1 = 0, lds2 = 0, lds2s = 0;   // their dynamic LDS bytes (lds2s: stacking)
    int64_t nb = 0;                // buckets per channel
    size_t cbytes = 0, rbytes = 0; // complex / real element bytes
    // device memory (per-channel arrays hold max_channels entries)
    Partial* partials = nullptr;
    Scalars* scalars = nullptr;
    WorkList* worklist = nullptr;
    int64_t* row_off = nullptr;    // channel table: [max_channels + 1] row offsets, then
    double* freq = nullptr;        // [max_channels] frequencies
    // pinned host staging of the channel table; staged_ev marks when the device has copied it
    void* staging = nullptr;
    hipEvent_t staged_ev = nullptr;
    bool staged_pending = false;
    // a second pinned table for calls captured into a HIP graph: the graph's copy node reads
    // it at every replay, so eager calls never write it
    void* staging_graph = nullptr;
    uint32_t *counts = nullptr, *offsets = nullptr, *tile_sums = nullptr;
    uint8_t *occ = nullptr, *plane_occ = nullptr;
    uint16_t* sflags = nullptr;    // stacking strip flags: [max_channels][nw][n >> lr2]
    int lr2 = 3;                   // log2 of the stacking pass's base radix
    uint32_t* list = nullptr;      // work list of occupied strips (heavy ones split into parts)
    uint32_t* list_aux = nullptr;  // each entry's part word
    uint32_t list_cap = 0;
    uint32_t* big = nullptr;       // the origin sort's big buckets (listed by k_occupancy)
    uint32_t big_cap = 0;          // rows / kBigBucket + 1 when the plan origin-sorts, else 0
    double2* split_acc = nullptr;  // float64 sums of split strips (zero between calls)
    uint32_t* split_done = nullptr;
    int persist_blocks = 256;      // work-groups of the persistent gridding kernel
    // the allocation-free entry point's transient plans: the channel table is written by a
    // kernel (no pinned staging), and no strip is split (no split-sum slots to keep zero)
    bool direct_channels = false;
    bool no_split = false;
    uint32_t *key = nullptr, *rank = nullptr, *rec_cell = nullptr, *rec_cell2 = nullptr;
    uint32_t* rec_idx = nullptr;   // input row of each record (prediction)
    void *rec = nullptr, *rec2 = nullptr, *inter = nullptr;   // records by bucket; by (bucket, origin)
    void *tw = nullptr, *inv_taper = nullptr, *kbc = nullptr;
    void *kbw = nullptr, *rec_w = nullptr, *rec_w2 = nullptr;   // w-kernel: polynomials, row offsets
    void* image_t = nullptr;       // the stacking pass's column-major images
    int64_t device_bytes = 0;
    std::vector<void*> allocations;
    // timing
    bool timing = false;
    std::vector<std::array<hipEvent_t, WSIMG_N_KERNELS + 1>> pending;
    std::vector<std::array<hipEvent_t, WSIMG_N_KERNELS + 1>> spare;
    wsimg_timing totals{};
};

namespace {

wsimg_status dev_alloc(wsimg_plan* pl, void** out, size_t bytes, const char* what) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        char buf[160];
        snprintf(buf, sizeof buf, "hipMalloc(%s, %zu bytes): %s", what, bytes, hipGetErrorString(e));
        return fail(e == hipErrorOutOfMemory ? WSIMG_E_NOMEM : WSIMG_E_HIP, buf);
    }
    pl->allocations.push_back(*out);
    pl->device_bytes += (int64_t)bytes;
    return WSIMG_OK;
}

inline unsigned blocks_for(int64_t count, int threads) {
    return (unsigned)((count + threads - 1) / threads);
}

void release(wsimg_plan* pl) {
    for (void* a : pl->allocations) (void)hipFree(a);
    pl->allocations.clear();
    if (pl->staging) (void)hipHostFree(pl->staging);
    pl->staging = nullptr;
    if (pl->staging_graph) (void)hipHostFree(pl->staging_graph);
    pl->staging_graph = nullptr;
    if (pl->staged_ev) (void)hipEventDestroy(pl->staged_ev);
    pl->staged_ev = nullptr;
    for (auto& ev : pl->pending) for (auto e : ev) (void)hipEventDestroy(e);
    for (auto& ev : pl->spare) for (auto e : ev) (void)hipEventDestroy(e);
    pl->pending.clear();
    pl->spare.clear();
}

// Reduction partials per channel for a call of nch channels (about 4096 blocks in all).
int parts_target(int nch) { return std::min(1024, std::max(16, 4096 / std::max(nch, 1))); }

constexpr int kMaxChannels = 65535;                 // the channel is a grid y index
constexpr int64_t kMaxBucketsTotal = int64_t(1) << 25;   // channels x buckets (x 64 counters)

wsimg_status validate_params(const wsimg_params* p, int64_t max_vis) {
    if (!p) return fail(WSIMG_E_INVALID, "params is NULL");
    if (p->precision != WSIMG_F32 && p->precision != WSIMG_F64)
        return fail(WSIMG_E_INVALID, "precision must be WSIMG_F32 or WSIMG_F64");
    if (!is_pow2(p->n) || p->n < 16 || p->n > 16384)
        return fail(WSIMG_E_INVALID, "n must be a power of two in [16, 16384]");
    if (p->n > 8192)
        return fail(WSIMG_E_UNSUPPORTED, "this build images n <= 8192");
    if (p->n_wplanes < 1 || p->n_wplanes > (int)kPlaneTab)
        return fail(WSIMG_E_INVALID, "n_wplanes must be in [1, 4096]");
    if (p->support < 3 || p->support > kMaxSupport || (p->support & 1) == 0 || p->support >= p->n)
        return fail(WSIMG_E_INVALID, "support must be odd, in [3, 15] and below n");
    if (!(p->pixel_rad > 0.0) || !std::isfinite(p->pixel_rad))
        return fail(WSIMG_E_INVALID, "pixel_rad must be finite and > 0");
    const double lmax = 0.5 * p->n * p->pixel_rad;
    if (!(2.0 * lmax * lmax < 1.0))
        return fail(WSIMG_E_INVALID, "field too wide: a corner pixel has l^2 + m^2 >= 1");
    if (!std::isfinite(p->beta)) return fail(WSIMG_E_INVALID, "beta must be finite");
    if ((p->flags & ~(WSIMG_FIXED_WRANGE | WSIMG_UNNORMALIZED | WSIMG_FOLD_W | WSIMG_PAD2 | WSIMG_COMPLEX_OUT)) != 0)
        return fail(WSIMG_E_INVALID, "unknown flags set");
    if (p->w_support != 0 &&
        (p->w_support < 3 || p->w_support > (uint32_t)kMaxSupport || (p->w_support & 1u) == 0 ||
         (int64_t)p->w_support >= (int64_t)p->n_wplanes))
        return fail(WSIMG_E_INVALID, "w_support must be 0, or odd in [3, 15] and below n_wplanes");
    if ((p->flags & WSIMG_PAD2) && p->n > 4096)
        return fail(WSIMG_E_UNSUPPORTED, "a padded grid is at most 8192 cells: n <= 4096 with WSIMG_PAD2");
    if (p->flags & WSIMG_FIXED_WRANGE) {
        if (!std::isfinite(p->w_lo) || !std::isfinite(p->w_hi) || p->w_lo > p->w_hi)
            return fail(WSIMG_E_INVALID, "fixed w range must be finite with w_lo <= w_hi");
    }
    if (max_vis < 0 || max_vis > 4294967294LL)
        return fail(WSIMG_E_INVALID, "max_vis must be in [0, 4294967294]");
    return WSIMG_OK;
}

template <typename R>
wsimg_status upload_tables(wsimg_plan* pl) {
    using C = typename Cx<R>::T;
    const int n = pl->g.n, n_img = pl->g.n_img, W = pl->p.support;
    const host::ld beta = (host::ld)pl->p.beta;
    const int deg = KbDeg<R>::value;
    std::vector<host::ld> coef = host::kb_tap_polynomials(W, beta, deg);
    std::vector<R> hc(coef.size());
    for (size_t i = 0; i < coef.size(); ++i) hc[i] = (R)coef[i];
    std::vector<host::ld> taper = host::inverse_taper(n_img, n, W, beta);
    std::vector<R> ht(n_img);
    for (int i = 0; i < n_img; ++i) ht[i] = (R)taper[i];
    std::vector<host::ld> tre, tim;
    host::twiddles(n, tre, tim);
    std::vector<C> htw(n);
    for (int i = 0; i < n; ++i) { htw[i].x = (R)tre[i]; htw[i].y = (R)tim[i]; }
    WS_HIP(hipMemcpy(pl->kbc, hc.data(), hc.size() * sizeof(R), hipMemcpyHostToDevice));
    if (pl->g.wsup) {      // the w-kernel's tap polynomials
        std::vector<host::ld> cw = host::kb_tap_polynomials((int)pl->g.wsup, (host::ld)pl->g.wbeta, deg);
        std::vector<R> hw(cw.size());
        for (size_t i = 0; i < cw.size(); ++i) hw[i] = (R)cw[i];
        WS_HIP(hipMemcpy(pl->kbw, hw.data(), hw.size() * sizeof(R), hipMemcpyHostToDevice));
    }
    WS_HIP(hipMemcpy(pl->inv_taper, ht.data(), ht.size() * sizeof(R), hipMemcpyHostToDevice));
    WS_HIP(hipMemcpy(pl->tw, htw.data(), htw.size() * sizeof(C), hipMemcpyHostToDevice));
    return WSIMG_OK;
}

// Fix the work-group shapes of a (precision, n) plan (host arithmetic only, no HIP call).
template <typename R, int LOG2N>
wsimg_status fill_shape(wsimg_plan* pl) {
    using SH = Shape<R, LOG2N>;
    Geom& g = pl->g;
    g.H = SH::H; g.log2H = Log2Of<SH::H>::value_any; g.S = SH::N / SH::H;
    g.B = SH::B; g.log2B = Log2Of<SH::B>::value_any; g.NB = SH::N / SH::B;
    pl->nt1 = SH::NT1;
    pl->nt2 = SH::NT2;
    pl->nt2a = SH::NT2A;
    pl->ba = SH::BA;
    pl->bs = SH::BS;
    pl->lds1 = SH::LDS1_BYTES;
    pl->lds2 = SH::LDS2_BYTES;
    pl->lds2s = SH::LDS2S_BYTES;
    pl->lr2 = SH::LR2;
    return WSIMG_OK;
}

// Raise the dynamic-LDS limits of a (precision, n) plan's kernels to the plan's sizes.
template <typename R, int LOG2N>
wsimg_status set_lds_limits(wsimg_plan* pl) {
    using SH = Shape<R, LOG2N>;
    WS_HIP(hipFuncSetAttribute((const void*)k_key<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kKeyLdsBytes));
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_rows<R, LOG2N, 7>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_rows<R, LOG2N, 9>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_only<R, LOG2N, 9>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_rows<R, LOG2N, kMaxSupport>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_only<R, LOG2N, 7>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_only<R, LOG2N, kMaxSupport>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_cols_stack<R, LOG2N, false, false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds2s));
    WS_HIP(hipFuncSetAttribute((const void*)k_cols_stack<R, LOG2N, true, false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds2s));
    WS_HIP(hipFuncSetAttribute((const void*)k_cols_stack<R, LOG2N, false, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds2s));
    WS_HIP(hipFuncSetAttribute((const void*)k_cols_stack<R, LOG2N, true, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds2s));
    WS_HIP(hipFuncSetAttribute((const void*)k_adj_cols<R, LOG2N>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds2));
    const int lds_adj = (int)(SH::LDS1 * sizeof(typename Cx<R>::T));
    WS_HIP(hipFuncSetAttribute((const void*)k_adj_rows<R, LOG2N, 7>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_adj));
    WS_HIP(hipFuncSetAttribute((const void*)k_adj_rows<R, LOG2N, kMaxSupport>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_adj));
    return WSIMG_OK;
}

#define WS_LAUNCH_CHECK(what)                                                               \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess) return fail(WSIMG_E_HIP, std::string("launch ") + what + ": " + hipGetErrorString(e_)); \
    } while (0)

// The records are put in origin order inside each bucket (k_origin_sort) for the float plan,
// and for the float64 plan at 8192^2 only: below it the float64 sort (36-byte records) costs
// more than the longer runs save (4096^2 float64 5.28 ms without it, 5.42 ms with it), at
// 8192^2, where a record is walked once per grid row of its taps, it pays (90.7 -> 86.2 ms:
// gridding 47.5 -> 40.0 ms for a 3.1 ms sort).  Unsorted plans grid in bucket order.
// (Without the origin sort the 8192^2 float gridding took 34.4 ms against 17.6 ms.)
template <typename R> bool origin_sorted(int log2n) { return sizeof(R) == 4 || log2n == 13; }
bool origin_sorted_plan(bool f32, int log2n) { return f32 || log2n == 13; }

// WMAX: the support class the gridding registers are sized for (W <= 7, else W <= 15).
template <typename R, int LOG2N, int WMAX>
wsimg_status launch_grid_w(wsimg_plan* pl, int nch, bool fft, void* out) {
    using C = typename Cx<R>::T;
    const Geom g = pl->g;
    const bool sorted = origin_sorted<R>(LOG2N);
    const uint32_t* rc = sorted ? pl->rec_cell2 : pl->rec_cell;
    const void* rr = sorted ? pl->rec2 : pl->rec;
    const R* recw = g.wsup ? (const R*)(sorted ? pl->rec_w2 : pl->rec_w) : nullptr;
    if (fft) {
        hipLaunchKernelGGL((k_grid_rows<R, LOG2N, WMAX>), dim3((unsigned)pl->persist_blocks), dim3(pl->nt1),
                           pl->lds1, pl->stream, g, pl->worklist, pl->list, pl->list_aux, pl->list_cap,
                           pl->offsets, rc, rr, (const R*)pl->kbc, (const C*)pl->tw,
                           (C*)out, pl->split_acc, pl->split_done, (const R*)pl->kbw, recw);
    } else {
        hipLaunchKernelGGL((k_grid_only<R, LOG2N, WMAX>), dim3((unsigned)(g.nw * g.S), (unsigned)nch),
                           dim3(pl->nt1), pl->lds1, pl->stream, g, pl->offsets, pl->occ, rc,
                           rr, (const R*)pl->kbc, (C*)out, (const R*)pl->kbw, recw);
    }
    WS_LAUNCH_CHECK("grid_rows");
    return WSIMG_OK;
}

template <typename R, int LOG2N>
wsimg_status launch_grid_rows(wsimg_plan* pl, int nch, bool fft, void* out) {
    // register classes of the gridding walk: supports up to 7, exactly 9, up to 15
    if (pl->g.support <= 7) return launch_grid_w<R, LOG2N, 7>(pl, nch, fft, out);
    if (pl->g.support == 9) return launch_grid_w<R, LOG2N, 9>(pl, nch, fft, out);
    return launch_grid_w<R, LOG2N, kMaxSupport>(pl, nch, fft, out);
}

template <typename R, int LOG2N>
wsimg_status launch_cols(wsimg_plan* pl, int nch, void* image) {
    using C = typename Cx<R>::T;
    const Geom g = pl->g;
    static_assert(Shape<R, LOG2N>::E2 <= 16, "stacking strip flags hold 16 bits");
    const int64_t nflags = (int64_t)nch * g.nw * (g.n >> pl->lr2);
    hipLaunchKernelGGL(k_stack_flags, dim3(blocks_for(nflags, 256)), dim3(256), 0, pl->stream, g, nch, pl->lr2,
                       (const uint8_t*)pl->occ, pl->sflags);
    WS_LAUNCH_CHECK("stack_flags");
    const dim3 grid((unsigned)(g.n_img / pl->bs), (unsigned)nch);
    auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(pl->nt2), pl->lds2s, pl->stream, g, pl->scalars, pl->sflags,
                           pl->plane_occ, (const C*)pl->inter, (const C*)pl->tw, (const R*)pl->inv_taper,
                           (R*)pl->image_t);
    };
    const bool cplx = (pl->p.flags & WSIMG_COMPLEX_OUT) != 0;
    if (g.crop > 0) {
        if (cplx) launch(k_cols_stack<R, LOG2N, true, true>);
        else launch(k_cols_stack<R, LOG2N, true, false>);
    } else {
        if (cplx) launch(k_cols_stack<R, LOG2N, false, true>);
        else launch(k_cols_stack<R, LOG2N, false, false>);
    }
    WS_LAUNCH_CHECK("cols_stack");
    // the column-major image -> the caller's row-major image
    const unsigned tiles = (unsigned)((g.n_img + 63) / 64);
    if (cplx)
        hipLaunchKernelGGL(k_transpose<C>, dim3(tiles, tiles, (unsigned)nch), dim3(256), 0, pl->stream, g.n_img,
                           (const C*)pl->image_t, (C*)image);
    else
        hipLaunchKernelGGL(k_transpose<R>, dim3(tiles, tiles, (unsigned)nch), dim3(256), 0, pl->stream, g.n_img,
                           (const R*)pl->image_t, (R*)image);
    WS_LAUNCH_CHECK("transpose");
    return WSIMG_OK;
}

// Call F<R, LOG2N>(args...) for the plan's image size (n = 16 .. 8192).
#define WS_SIZE_DISPATCH(R, log2n, FN, ...)                                                  \
    switch (log2n) {                                                                         \
        case 4: return FN<R, 4>(__VA_ARGS__);                                                \
        case 5: return FN<R, 5>(__VA_ARGS__);                                                \
        case 6: return FN<R, 6>(__VA_ARGS__);                                                \
        case 7: return FN<R, 7>(__VA_ARGS__);                                                \
        case 8: return FN<R, 8>(__VA_ARGS__);                                                \
        case 9: return FN<R, 9>(__VA_ARGS__);                                                \
        case 10: return FN<R, 10>(__VA_ARGS__);                                              \
        case 11: return FN<R, 11>(__VA_ARGS__);                                              \
        case 12: return FN<R, 12>(__VA_ARGS__);                                              \
        case 13: return FN<R, 13>(__VA_ARGS__);                                              \
        default: return fail(WSIMG_E_UNSUPPORTED, "image size outside 16..8192");             \
    }

template <typename R> wsimg_status shape_of(wsimg_plan* pl) { WS_SIZE_DISPATCH(R, pl->g.log2n, fill_shape, pl) }
template <typename R> wsimg_status lds_limits(wsimg_plan* pl) { WS_SIZE_DISPATCH(R, pl->g.log2n, set_lds_limits, pl) }
template <typename R> wsimg_status grid_rows(wsimg_plan* pl, int nch, bool fft, void* out) {
    WS_SIZE_DISPATCH(R, pl->g.log2n, launch_grid_rows, pl, nch, fft, out)
}
template <typename R> wsimg_status cols_stack(wsimg_plan* pl, int nch, void* image) {
    WS_SIZE_DISPATCH(R, pl->g.log2n, launch_cols, pl, nch, image)
}

// Prediction: column pass (image -> intermediate), then the persistent row pass + degridding.
template <typename R, int LOG2N, int WMAX>
wsimg_status launch_adj_rows_w(wsimg_plan* pl, int nch, void* vis_out) {
    using C = typename Cx<R>::T;
    const size_t lds = (size_t)Shape<R, LOG2N>::LDS1 * sizeof(C);
    hipLaunchKernelGGL((k_adj_rows<R, LOG2N, WMAX>), dim3((unsigned)pl->persist_blocks), dim3(pl->nt1), lds,
                       pl->stream, pl->g, pl->worklist, pl->list, pl->list_aux, pl->list_cap, pl->offsets,
                       pl->rec_cell,
                       (const void*)pl->rec, (const uint32_t*)pl->rec_idx, (const R*)pl->kbc,
                       (const C*)pl->tw, (const C*)pl->inter, (C*)vis_out);
    WS_LAUNCH_CHECK("adj_rows");
    return WSIMG_OK;
}

template <typename R, int LOG2N>
wsimg_status launch_predict(wsimg_plan* pl, int nch, const void* image, void* vis_out) {
    using C = typename Cx<R>::T;
    const Geom g = pl->g;
    hipLaunchKernelGGL((k_adj_cols<R, LOG2N>), dim3((unsigned)g.NB, (unsigned)nch), dim3(pl->nt2a), pl->lds2,
                       pl->stream, g, pl->scalars, pl->occ, pl->plane_occ, (const R*)image, (const C*)pl->tw,
                       (const R*)pl->inv_taper, (C*)pl->inter);
    WS_LAUNCH_CHECK("adj_cols");
    return g.support <= 7 ? launch_adj_rows_w<R, LOG2N, 7>(pl, nch, vis_out)
                          : launch_adj_rows_w<R, LOG2N, kMaxSupport>(pl, nch, vis_out);
}

template <typename R> wsimg_status predict_passes(wsimg_plan* pl, int nch, const void* image, void* vis_out) {
    WS_SIZE_DISPATCH(R, pl->g.log2n, launch_predict, pl, nch, image, vis_out)
}

// A call's channels: counts and frequencies as passed (host), with their totals.
struct Batch {
    int nch = 0;
    const int64_t* counts = nullptr;
    const double* freqs = nullptr;
    int64_t total = 0, max_count = 0;
};

wsimg_status validate_call(wsimg_plan* pl, int nch, const int64_t* counts, const double* freqs,
                           const double* uvw, const void* vis, const void* weights, void* out, Batch& bt) {
    if (!pl) return fail(WSIMG_E_INVALID, "plan is NULL");
    if (nch < 1 || nch > pl->max_channels)
        return fail(WSIMG_E_INVALID, "n_channels must be in [1, the plan's max_channels]");
    if (!counts || !freqs) return fail(WSIMG_E_INVALID, "row_counts or freqs_hz is NULL");
    int64_t total = 0, mx = 0;
    for (int c = 0; c < nch; ++c) {
        if (counts[c] < 0) return fail(WSIMG_E_INVALID, "n_vis < 0");
        if (counts[c] > pl->max_vis || total > pl->max_vis - counts[c])
            return fail(WSIMG_E_CAPACITY, "n_vis exceeds the plan's max_vis");
        total += counts[c];
        mx = std::max(mx, counts[c]);
        if (!(freqs[c] > 0.0) || !std::isfinite(freqs[c]))
            return fail(WSIMG_E_INVALID, "freq_hz must be finite and > 0");
    }
    if (total > 0 && (!uvw || !vis || !weights)) return fail(WSIMG_E_INVALID, "input pointer is NULL");
    if (!out) return fail(WSIMG_E_INVALID, "output pointer is NULL");
    bt.nch = nch; bt.counts = counts; bt.freqs = freqs; bt.total = total; bt.max_count = mx;
    return WSIMG_OK;
}

// True while the plan's stream is being captured into a HIP graph.
bool capturing(const wsimg_plan* pl) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(pl->stream, &cs) != hipSuccess) return false;
    return cs == hipStreamCaptureStatusActive;
}

// Channel table -> pinned staging -> device, on the plan's stream.  The staging buffer is
// rewritten only after the device has copied the previous call's table.  Under capture the
// table goes to the graph's own buffer, with no host wait.
wsimg_status upload_channels(wsimg_plan* pl, const Batch& bt) {
    if (pl->direct_channels) {
        if (bt.nch != 1) return fail(WSIMG_E_INVALID, "a direct channel table holds one channel");
        hipLaunchKernelGGL(k_set_channel, dim3(1), dim3(64), 0, pl->stream, pl->row_off, pl->freq,
                           bt.counts[0], bt.freqs[0]);
        WS_LAUNCH_CHECK("set_channel");
        return WSIMG_OK;
    }
    const bool cap = capturing(pl);
    if (!cap && pl->staged_pending) {
        WS_HIP(hipEventSynchronize(pl->staged_ev));
        pl->staged_pending = false;
    }
    int64_t* ro = static_cast<int64_t*>(cap ? pl->staging_graph : pl->staging);
    double* fq = reinterpret_cast<double*>(ro + (pl->max_channels + 1));
    ro[0] = 0;
    for (int c = 0; c < bt.nch; ++c) { ro[c + 1] = ro[c] + bt.counts[c]; fq[c] = bt.freqs[c]; }
    WS_HIP(hipMemcpyAsync(pl->row_off, ro, sizeof(int64_t) * (bt.nch + 1), hipMemcpyHostToDevice, pl->stream));
    WS_HIP(hipMemcpyAsync(pl->freq, fq, sizeof(double) * bt.nch, hipMemcpyHostToDevice, pl->stream));
    if (cap) return WSIMG_OK;
    WS_HIP(hipEventRecord(pl->staged_ev, pl->stream));
    pl->staged_pending = true;
    return WSIMG_OK;
}

struct Stamp {
    wsimg_plan* pl;
    std::array<hipEvent_t, WSIMG_N_KERNELS + 1>* ev = nullptr;
    explicit Stamp(wsimg_plan* p) : pl(p) {}
    wsimg_status begin() {
        if (!pl->timing || capturing(pl)) return WSIMG_OK;
        std::array<hipEvent_t, WSIMG_N_KERNELS + 1> e{};
        if (!pl->spare.empty()) { e = pl->spare.back(); pl->spare.pop_back(); }
        else for (auto& x : e) WS_HIP(hipEventCreate(&x));
        pl->pending.push_back(e);
        ev = &pl->pending.back();
        WS_HIP(hipEventRecord((*ev)[0], pl->stream));
        return WSIMG_OK;
    }
    // every stage is stamped, also one that launched nothing, so elapsed times line up
    wsimg_status after(int stage) {
        if (!ev) return WSIMG_OK;
        WS_HIP(hipEventRecord((*ev)[stage + 1], pl->stream));
        return WSIMG_OK;
    }
};

// Stages shared by wsimg_image and wsimg_grid: counters, plane ranges, bucket sort.
// vis == nullptr: the sort for a prediction (records carry positions and their input rows,
// and need no origin order).
template <typename R>
wsimg_status run_sort(wsimg_plan* pl, Stamp& st, const Batch& bt, const double* uvw, const void* vis,
                      const void* wts) {
    const bool predict = vis == nullptr;
    using C = typename Cx<R>::T;
    const Geom g = pl->g;
    hipStream_t s = pl->stream;
    const int nch = bt.nch;
    const int64_t nbk = pl->nb * nch;
    const int64_t ncnt = nbk * kReplicas;
    const Chan ch{pl->row_off, pl->freq};
    if (auto r = upload_channels(pl, bt)) return r;
    hipLaunchKernelGGL(k_fill_u32, dim3(std::min<int64_t>(blocks_for(ncnt, 256), 8192)), dim3(256), 0, s,
                       pl->counts, ncnt, 0u);
    WS_LAUNCH_CHECK("fill");
    if (auto r = st.after(0)) return r;

    const int64_t M = bt.max_count;
    const int64_t chunk = std::max<int64_t>(1, (M + parts_target(nch) - 1) / parts_target(nch));
    const int nparts = M > 0 ? (int)((M + chunk - 1) / chunk) : 0;
    if (nparts > 0) {
        hipLaunchKernelGGL((k_reduce<R>), dim3(nparts, nch), dim3(256), 0, s, ch, chunk, nparts, uvw,
                           (const R*)wts, g, pl->partials);
        WS_LAUNCH_CHECK("reduce");
    }
    hipLaunchKernelGGL(k_finalize, dim3(nch), dim3(256), 0, s, nparts, pl->partials, g, ch, pl->scalars,
                       pl->worklist);
    WS_LAUNCH_CHECK("finalize");
    if (auto r = st.after(1)) return r;

    if (M > 0) {
        hipLaunchKernelGGL((k_key<R>), dim3(blocks_for(M, kKeyRows), nch), dim3(kKeyThreads), kKeyLdsBytes, s, ch, uvw, (const R*)wts,
                           g, pl->scalars, pl->key, pl->rank, pl->counts);
        WS_LAUNCH_CHECK("key");
    }
    if (auto r = st.after(2)) return r;

    const int ntiles = (int)((ncnt + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, ncnt, pl->counts, pl->tile_sums);
    WS_LAUNCH_CHECK("scan_tiles");
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, ntiles, pl->tile_sums);
    WS_LAUNCH_CHECK("scan_top");
    hipLaunchKernelGGL(k_scan_down, dim3(ntiles), dim3(256), 0, s, ncnt, pl->counts, pl->tile_sums, pl->offsets);
    WS_LAUNCH_CHECK("scan_down");
    // each gridding work-group's share of the call's record visits (a row's taps reach about
    // (W + H - 2) / H + 1 strips)
    const int64_t visits = bt.total * (int64_t)((g.support + g.H - 2) / g.H + 1);
    // a strip gridded from several planes' rows (the w-kernel) is not split into parts
    const int64_t share = (pl->no_split || g.wsup) ? int64_t(0x3FFFFFFF)
                                       : std::max<int64_t>(kMinPart, visits / std::max(1, pl->persist_blocks));
    const bool osort = M > 0 && !predict && origin_sorted<R>(g.log2n) && pl->big_cap > 0;
    hipLaunchKernelGGL(k_occupancy, dim3(blocks_for(nbk, 256)), dim3(256), 0, s, nch, pl->offsets, g,
                       pl->occ, pl->plane_occ, pl->list, pl->list_aux, pl->list_cap,
                       (uint32_t)std::min<int64_t>(share, 0x3FFFFFFF), pl->scalars, pl->worklist,
                       osort ? pl->big : nullptr);
    WS_LAUNCH_CHECK("occupancy");
    if (auto r = st.after(3)) return r;

    if (M > 0) {
        hipLaunchKernelGGL((k_scatter<R, R>), dim3(blocks_for(M, kScatterThreads), nch), dim3(kScatterThreads), 0, s, ch, uvw,
                           (const C*)vis, (const R*)wts, g, pl->key, pl->rank, pl->offsets,
                           pl->rec_cell, pl->rec, predict ? pl->rec_idx : nullptr, pl->scalars,
                           g.wsup ? (R*)pl->rec_w : nullptr);
        WS_LAUNCH_CHECK("scatter");
    }
    if (auto r = st.after(4)) return r;

    if (osort) {
        // the first big_cap blocks take the listed big buckets, the rest every bucket of every channel
        hipLaunchKernelGGL((k_origin_sort<R>), dim3((unsigned)(pl->big_cap + nbk)), dim3(kSortThreads), 0, s, g,
                           pl->offsets, pl->rec_cell, (const void*)pl->rec, pl->rec_cell2, pl->rec2,
                           g.wsup ? (const R*)pl->rec_w : nullptr, g.wsup ? (R*)pl->rec_w2 : nullptr,
                           (const uint32_t*)pl->big, pl->big_cap, (const WorkList*)pl->worklist);
        WS_LAUNCH_CHECK("origin_sort");
    }
    if (auto r = st.after(5)) return r;
    return WSIMG_OK;
}

template <typename R>
wsimg_status run_image(wsimg_plan* pl, const Batch& bt, const double* uvw, const void* vis, const void* wts,
                       void* image, bool grid_only) {
    Stamp st(pl);
    if (auto r = st.begin()) return r;
    if (auto r = run_sort<R>(pl, st, bt, uvw, vis, wts)) return r;
    if (grid_only) {
        if (auto r = grid_rows<R>(pl, bt.nch, false, image)) return r;
        if (auto r = st.after(6)) return r;
        if (auto r = st.after(7)) return r;
        return WSIMG_OK;
    }
    if (auto r = grid_rows<R>(pl, bt.nch, true, pl->inter)) return r;
    if (auto r = st.after(6)) return r;
    if (auto r = cols_stack<R>(pl, bt.nch, image)) return r;
    if (auto r = st.after(7)) return r;
    return WSIMG_OK;
}

wsimg_status finish_call(wsimg_plan* pl, int nch, wsimg_stats* stats, bool empty_is_error = true) {
    if (!stats) return WSIMG_OK;
    std::vector<Scalars> h((size_t)nch);
    WS_HIP(hipMemcpyAsync(h.data(), pl->scalars, sizeof(Scalars) * nch, hipMemcpyDeviceToHost, pl->stream));
    WS_HIP(hipStreamSynchronize(pl->stream));
    bool empty = false;
    for (int c = 0; c < nch; ++c) {
        wsimg_stats& o = stats[c];
        o.n_in = (int64_t)h[c].n_in;
        o.n_gridded = (int64_t)h[c].n_kept;
        o.n_dropped = (int64_t)(h[c].n_in - h[c].n_kept);
        o.sum_w = h[c].sum_w;
        o.w_lo = h[c].w_lo;
        o.w_hi = h[c].w_hi;
        o.n_strips_occupied = (int64_t)h[c].n_occ;
        o.n_planes_occupied = (int64_t)h[c].n_planes;
        if (!(h[c].sum_w != 0.0)) empty = true;
    }
    if (empty && empty_is_error) return fail(WSIMG_E_EMPTY, "the kept visibilities of a channel have zero total weight");
    return WSIMG_OK;
}

wsimg_status dispatch(wsimg_plan* pl, int nch, const int64_t* counts, const double* uvw, const void* vis,
                      const void* wts, const double* freqs, void* out, wsimg_stats* stats, bool grid_only) {
    Batch bt;
    if (auto r = validate_call(pl, nch, counts, freqs, uvw, vis, wts, out, bt)) return r;
    if (stats && capturing(pl)) return fail(WSIMG_E_INVALID, "stats need a host wait: not under graph capture");
    WS_HIP(hipSetDevice(pl->device));
    wsimg_status r = pl->p.precision == WSIMG_F32
                         ? run_image<float>(pl, bt, uvw, vis, wts, out, grid_only)
                         : run_image<double>(pl, bt, uvw, vis, wts, out, grid_only);
    if (r) return r;
    return finish_call(pl, nch, stats);
}

template <typename R>
wsimg_status run_predict(wsimg_plan* pl, const Batch& bt, const double* uvw, const void* wts, const void* image,
                         void* vis_out) {
    Stamp st(pl);
    if (auto r = st.begin()) return r;
    if (auto r = run_sort<R>(pl, st, bt, uvw, nullptr, wts)) return r;
    const int64_t words = bt.total * (int64_t)(2 * sizeof(R) / 4);
    if (words > 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(std::min<int64_t>(blocks_for(words, 256), 8192)), dim3(256), 0,
                           pl->stream, (uint32_t*)vis_out, words, 0u);
        WS_LAUNCH_CHECK("zero visibilities");
    }
    if (auto r = st.after(5)) return r;
    if (bt.total > 0) {
        if (auto r = predict_passes<R>(pl, bt.nch, image, vis_out)) return r;
    }
    if (auto r = st.after(6)) return r;
    if (auto r = st.after(7)) return r;
    return WSIMG_OK;
}

wsimg_status dispatch_predict(wsimg_plan* pl, int64_t n_vis, const double* uvw, const void* wts, double freq,
                              const void* image, void* vis_out, wsimg_stats* stats) {
    Batch bt;
    if (auto r = validate_call(pl, 1, &n_vis, &freq, uvw, wts, wts, vis_out, bt)) return r;
    if (!image) return fail(WSIMG_E_INVALID, "image pointer is NULL");
    if (pl->p.flags & WSIMG_COMPLEX_OUT)
        return fail(WSIMG_E_INVALID, "wsimg_predict takes a real image: the plan has WSIMG_COMPLEX_OUT");
    if (pl->g.wsup)
        return fail(WSIMG_E_UNSUPPORTED, "wsimg_predict is the transpose of nearest-plane imaging (w_support 0)");
    if (stats && capturing(pl)) return fail(WSIMG_E_INVALID, "stats need a host wait: not under graph capture");
    WS_HIP(hipSetDevice(pl->device));
    wsimg_status r = pl->p.precision == WSIMG_F32 ? run_predict<float>(pl, bt, uvw, wts, image, vis_out)
                                                  : run_predict<double>(pl, bt, uvw, wts, image, vis_out);
    if (r) return r;
    return finish_call(pl, 1, stats, false);
}

// Rows of slack after the last row in every row-indexed scratch buffer (keys, ranks, records,
// record rows): a read one record past the last one stays inside the allocation.  (A buffer
// of exactly 16 * max_vis bytes can end on an allocation-granule boundary, e.g. 32 MiB for
// 2^21 float records, where one 16-byte record past its end is unmapped memory.)
constexpr size_t kRowSlack = 256;

// Geometry and work-group shapes of a plan from its parameters: host arithmetic only.
wsimg_status plan_geometry(wsimg_plan* pl, const wsimg_params* p, int64_t max_vis, int max_channels) {
    if (auto r = validate_params(p, max_vis)) return r;
    if (max_channels < 1 || max_channels > kMaxChannels)
        return fail(WSIMG_E_INVALID, "max_channels must be in [1, 65535]");
    pl->p = *p;
    if (!(pl->p.beta > 0.0)) pl->p.beta = 2.34 * pl->p.support;
    pl->max_vis = max_vis;
    pl->max_channels = max_channels;
    const bool f32 = p->precision == WSIMG_F32;
    pl->rbytes = f32 ? 4 : 8;
    pl->cbytes = 2 * pl->rbytes;
    const int n_img = p->n;
    const int n = (p->flags & WSIMG_PAD2) ? 2 * n_img : n_img;      // grid side
    Geom& g = pl->g;
    g.n = n; g.log2n = ilog2(n); g.nw = p->n_wplanes; g.support = p->support; g.half = (p->support - 1) / 2;
    g.n_img = n_img;
    g.crop = (n - n_img) / 2;
    g.plane_elems = (size_t)n * (size_t)n_img;
    g.du = 1.0 / ((double)n * p->pixel_rad);
    g.half_n = (double)n / 2.0;
    g.pixel = p->pixel_rad;
    g.fixed_range = (p->flags & WSIMG_FIXED_WRANGE) ? 1 : 0;
    g.unnormalized = (p->flags & WSIMG_UNNORMALIZED) ? 1 : 0;
    g.fold_w = (p->flags & WSIMG_FOLD_W) ? 1 : 0;
    g.wsup = (int)p->w_support;
    g.whalf = g.wsup ? (g.wsup - 1) / 2 : 0;
    g.wbeta = 2.34 * g.wsup;
    g.wscale = g.wsup ? (double)((host::ld)g.wsup / host::bessel_i0((host::ld)g.wbeta)) : 0.0;
    g.w_lo_fixed = p->w_lo; g.w_hi_fixed = p->w_hi;
    if (auto r = f32 ? shape_of<float>(pl) : shape_of<double>(pl)) return r;
    pl->nb = (int64_t)g.nw * g.S;
    g.nb1 = (int)pl->nb;
    g.NB = n_img / pl->ba;          // prediction column blocks cover the image's columns only
    if (pl->nb * max_channels > kMaxBucketsTotal)
        return fail(WSIMG_E_UNSUPPORTED, "max_channels x n_wplanes x strips exceeds 2^25 sort buckets");
    pl->list_cap = (uint32_t)((size_t)pl->nb * max_channels + (size_t)kMaxSplit * kMaxParts);
    // a big bucket holds more than kBigBucket of the call's rows, so there are fewer than this
    pl->big_cap = origin_sorted_plan(f32, g.log2n)
                      ? (uint32_t)(((size_t)std::max<int64_t>(max_vis, 1) + kRowSlack) / kBigBucket + 1) : 0u;
    return WSIMG_OK;
}

// Every device allocation of a plan, in order: f(address of the plan member, bytes, name).
template <typename F>
wsimg_status for_each_allocation(wsimg_plan* pl, F&& f) {
    const Geom& g = pl->g;
    const bool f32 = pl->p.precision == WSIMG_F32;
    const size_t rows = (size_t)std::max<int64_t>(pl->max_vis, 1) + kRowSlack;
    const size_t mc = (size_t)pl->max_channels;
    const size_t cells = (size_t)g.nw * g.plane_elems;
    const size_t nbt = (size_t)pl->nb * mc;
    size_t nparts_alloc = 0;
    for (int c = 1; c <= pl->max_channels; ++c) nparts_alloc = std::max(nparts_alloc, (size_t)c * parts_target(c));
    const bool sorted2 = origin_sorted_plan(f32, g.log2n);     // origin-ordered copies exist
    const size_t rec_bytes = f32 ? 16 : 32;
    wsimg_status r = WSIMG_OK;
#define WS_ALLOC(field, bytes, name) \
    if (!r) r = f((void**)&pl->field, (size_t)(bytes), name);
    WS_ALLOC(partials, sizeof(Partial) * nparts_alloc, "partials");
    WS_ALLOC(scalars, sizeof(Scalars) * mc, "scalars");
    WS_ALLOC(worklist, sizeof(WorkList), "work list counters");
    WS_ALLOC(row_off, sizeof(int64_t) * (mc + 1), "channel row offsets");
    WS_ALLOC(freq, sizeof(double) * mc, "channel frequencies");
    WS_ALLOC(counts, sizeof(uint32_t) * nbt * kReplicas, "counts");
    WS_ALLOC(offsets, sizeof(uint32_t) * (nbt * kReplicas + 1), "offsets");
    WS_ALLOC(tile_sums, sizeof(uint32_t) * ((nbt * kReplicas + kScanTile - 1) / kScanTile), "scan tiles");
    WS_ALLOC(occ, nbt, "occupancy");
    WS_ALLOC(list, sizeof(uint32_t) * pl->list_cap, "strip work list");
    WS_ALLOC(list_aux, sizeof(uint32_t) * pl->list_cap, "strip work list parts");
    WS_ALLOC(big, sizeof(uint32_t) * std::max<uint32_t>(pl->big_cap, 1), "big-bucket list");
    WS_ALLOC(split_acc, pl->no_split ? 256 : (size_t)kMaxSplit * pl->lds1, "split strip sums");
    WS_ALLOC(split_done, pl->no_split ? 256 : sizeof(uint32_t) * kMaxSplit, "split strip counters");
    WS_ALLOC(plane_occ, (size_t)g.nw * mc, "plane occupancy");
    WS_ALLOC(sflags, sizeof(uint16_t) * mc * g.nw * (size_t)(g.n >> pl->lr2), "stacking strip flags");
    WS_ALLOC(key, sizeof(uint32_t) * rows, "keys");
    WS_ALLOC(rank, sizeof(uint32_t) * rows, "ranks");
    WS_ALLOC(rec_cell, f32 ? 256 : sizeof(uint32_t) * rows, "record cells");
    WS_ALLOC(rec, rec_bytes * rows, "records");
    WS_ALLOC(rec_cell2, (f32 || !sorted2) ? 256 : sizeof(uint32_t) * rows, "record cells by origin");
    WS_ALLOC(rec_idx, sizeof(uint32_t) * rows, "record rows");
    WS_ALLOC(rec2, sorted2 ? rec_bytes * rows : 256, "records by origin");
    WS_ALLOC(inter, pl->cbytes * cells * mc, "row-transformed planes");
    WS_ALLOC(image_t, ((pl->p.flags & WSIMG_COMPLEX_OUT) ? pl->cbytes : pl->rbytes) * (size_t)g.n_img * g.n_img * mc,
             "column-major images");
    WS_ALLOC(tw, pl->cbytes * g.n, "twiddles");
    WS_ALLOC(inv_taper, pl->rbytes * g.n_img, "taper");
    WS_ALLOC(kbc, pl->rbytes * (size_t)pl->p.support * 17, "kernel polynomials");
    const bool wk = g.wsup != 0;
    WS_ALLOC(kbw, wk ? pl->rbytes * (size_t)g.wsup * 17 : 256, "w-kernel polynomials");
    WS_ALLOC(rec_w, wk ? pl->rbytes * rows : 256, "record w-offsets");
    WS_ALLOC(rec_w2, (wk && sorted2) ? pl->rbytes * rows : 256, "record w-offsets by origin");
#undef WS_ALLOC
    return r;
}

void fill_info(const wsimg_plan* plan, wsimg_plan_info* info) {
    info->n = plan->p.n;
    info->n_wplanes = plan->p.n_wplanes;
    info->support = plan->p.support;
    info->precision = plan->p.precision;
    info->strip_rows = plan->g.H;
    info->col_block = plan->g.B;
    info->n_buckets = plan->nb;
    info->max_vis = plan->max_vis;
    info->device_bytes = plan->device_bytes;
    info->max_channels = plan->max_channels;
    info->n_grid = plan->g.n;
    info->grid_threads = plan->nt1;
    info->stack_threads = plan->nt2;
    info->stack_cols = plan->bs;
    info->stack_radix = 1 << plan->lr2;
    info->lds_grid_bytes = (int64_t)plan->lds1;
    info->lds_stack_bytes = (int64_t)plan->lds2s;
    info->record_bytes = plan->p.precision == WSIMG_F32 ? 16 : 32;
    info->row_capacity = (int64_t)((size_t)std::max<int64_t>(plan->max_vis, 1) + kRowSlack);
    info->list_capacity = (int64_t)plan->list_cap;
}

wsimg_status create(wsimg_plan** out, const wsimg_params* p, int64_t max_vis, int max_channels,
                    void* hip_stream) {
    if (!out) return fail(WSIMG_E_INVALID, "out is NULL");
    *out = nullptr;
    wsimg_plan* pl = new (std::nothrow) wsimg_plan();
    if (!pl) return fail(WSIMG_E_NOMEM, "host allocation of the plan failed");
    if (auto r = plan_geometry(pl, p, max_vis, max_channels)) { delete pl; return r; }
    pl->stream = (hipStream_t)hip_stream;
    const bool f32 = p->precision == WSIMG_F32;
    {
        wsimg_status rs = f32 ? lds_limits<float>(pl) : lds_limits<double>(pl);
        if (rs) { delete pl; return rs; }
    }

    hipError_t he = hipGetDevice(&pl->device);
    if (he != hipSuccess) { delete pl; return fail(WSIMG_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he)); }
    int cus = 0;
    he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device);
    if (he != hipSuccess || cus <= 0) { delete pl; return fail(WSIMG_E_HIP, "hipDeviceGetAttribute(CU count) failed"); }
    // as many strip work-groups as fit at once: one per CU while the LDS strip exceeds 80 KB
    pl->persist_blocks = cus * std::max(1, (int)((160 * 1024) / std::max<size_t>(pl->lds1, 1)));

    wsimg_status r = for_each_allocation(pl, [pl](void** field, size_t bytes, const char* name) {
        return dev_alloc(pl, field, bytes, name);
    });
    const size_t mc = (size_t)max_channels;
    if (!r) {
        const size_t tb = sizeof(int64_t) * (mc + 1) + sizeof(double) * mc;
        hipError_t e = hipHostMalloc(&pl->staging, tb, hipHostMallocDefault);
        if (e != hipSuccess) { pl->staging = nullptr; r = fail(WSIMG_E_NOMEM, "hipHostMalloc(channel table) failed"); }
        if (!r) {
            e = hipHostMalloc(&pl->staging_graph, tb, hipHostMallocDefault);
            if (e != hipSuccess) { pl->staging_graph = nullptr; r = fail(WSIMG_E_NOMEM, "hipHostMalloc(graph table) failed"); }
        }
    }
    if (!r) {
        hipError_t e = hipEventCreateWithFlags(&pl->staged_ev, hipEventDisableTiming);
        if (e != hipSuccess) { pl->staged_ev = nullptr; r = fail(WSIMG_E_HIP, "hipEventCreate failed"); }
    }
    if (!r) r = f32 ? upload_tables<float>(pl) : upload_tables<double>(pl);
    if (!r) {
        hipError_t e = hipMemset(pl->split_acc, 0, (size_t)kMaxSplit * pl->lds1);
        if (e == hipSuccess) e = hipMemset(pl->split_done, 0, sizeof(uint32_t) * kMaxSplit);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) r = fail(WSIMG_E_HIP, std::string("clearing split slots: ") + hipGetErrorString(e));
    }
    if (r) { release(pl); delete pl; return r; }
    *out = pl;
    return WSIMG_OK;
}

// ---------------------------------------------------------------------------------------
// The allocation-free entry point: a transient plan whose scratch is carved from one static
// device array instead of hipMalloc'ed buffers.  Every GPU the library runs on holds its own
// copy of the array (from module load to process end).  In host code the array's name is
// only a stand-in for its device address, so the address of this device's copy is taken once
// per device with hipGetSymbolAddress (with that device current) and only that address is
// ever handed to kernels or copies.
constexpr size_t kStaticTableBytes = size_t(256) << 10;   // twiddles, taper, kernel polynomials
static_assert(WSIMG_NOALLOC_SCRATCH_BYTES > kStaticTableBytes, "static scratch too small");
static __device__ __align__(256) unsigned char scratch[WSIMG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
struct StaticScratch {
    void* ptr = nullptr;            // this device's copy of `scratch`
    bool tables_valid = false;      // the table region holds the tables of `key`
    double key[6] = {0, 0, 0, 0, 0, 0};
};
std::mutex g_scratch_mu;
StaticScratch g_scratch[kMaxDevices];

// The table key of a plan: every quantity upload_tables reads.
void table_key(const wsimg_plan* pl, double key[6]) {
    key[0] = pl->p.precision; key[1] = pl->g.n; key[2] = pl->g.n_img; key[3] = pl->p.support;
    key[4] = pl->p.beta; key[5] = 1.0 + pl->g.wsup;
}

template <typename R>
wsimg_status upload_tables_async(wsimg_plan* pl) {
    // the tables go out through pageable host vectors: wait for the copies before they die
    if (auto r = upload_tables<R>(pl)) return r;
    WS_HIP(hipStreamSynchronize(pl->stream));
    return WSIMG_OK;
}

wsimg_status image_noalloc(const wsimg_params* p, int64_t n_vis, const double* uvw, const void* vis,
                           const void* wts, double freq_hz, void* image_out, void* hip_stream,
                           wsimg_stats* stats) {
    if (n_vis < 0) return fail(WSIMG_E_INVALID, "n_vis < 0");
    wsimg_plan pl;
    if (auto r = plan_geometry(&pl, p, n_vis, 1)) return r;
    pl.direct_channels = true;
    pl.no_split = true;
    pl.stream = (hipStream_t)hip_stream;
    // sizes first (host arithmetic): the tables at the start of the array, the rest after them
    auto is_table = [&pl](void** field) {
        return field == &pl.tw || field == &pl.inv_taper || field == &pl.kbc || field == &pl.kbw;
    };
    size_t tab_need = 0, need = kStaticTableBytes;
    for_each_allocation(&pl, [&](void** field, size_t b, const char*) {
        (is_table(field) ? tab_need : need) += (std::max<size_t>(b, 256) + 255) & ~size_t(255);
        return WSIMG_OK;
    });
    if (tab_need > kStaticTableBytes || need > (size_t)WSIMG_NOALLOC_SCRATCH_BYTES) {
        char buf[200];
        snprintf(buf, sizeof buf, "wsimg_image_noalloc: this geometry and n_vis need %zu bytes of scratch; "
                 "the static scratch holds %zu", need + (tab_need > kStaticTableBytes ? tab_need : 0),
                 (size_t)WSIMG_NOALLOC_SCRATCH_BYTES);
        return fail(WSIMG_E_CAPACITY, buf);
    }
    if (n_vis > 0 && (!uvw || !vis || !wts)) return fail(WSIMG_E_INVALID, "input pointer is NULL");
    if (!image_out) return fail(WSIMG_E_INVALID, "output pointer is NULL");
    if (stats && capturing(&pl)) return fail(WSIMG_E_INVALID, "stats need a host wait: not under graph capture");
    WS_HIP(hipGetDevice(&pl.device));
    if (pl.device < 0 || pl.device >= kMaxDevices) return fail(WSIMG_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    StaticScratch& ss = g_scratch[pl.device];
    if (!ss.ptr) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(WSIMG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        ss.ptr = ptr;
    }
    const bool f32 = p->precision == WSIMG_F32;
    if (auto r = f32 ? lds_limits<float>(&pl) : lds_limits<double>(&pl)) return r;
    int cus = 0;
    WS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl.device));
    pl.persist_blocks = std::max(1, cus) * std::max(1, (int)((160 * 1024) / std::max<size_t>(pl.lds1, 1)));
    // carve
    unsigned char* base = static_cast<unsigned char*>(ss.ptr);
    size_t tab_off = 0, off = kStaticTableBytes;
    for_each_allocation(&pl, [&](void** field, size_t b, const char*) {
        const size_t sz = (std::max<size_t>(b, 256) + 255) & ~size_t(255);
        size_t& at = is_table(field) ? tab_off : off;
        *field = base + at;
        at += sz;
        return WSIMG_OK;
    });
    double key[6];
    table_key(&pl, key);
    if (!ss.tables_valid || std::memcmp(key, ss.key, sizeof key) != 0) {
        ss.tables_valid = false;
        if (auto r = f32 ? upload_tables_async<float>(&pl) : upload_tables_async<double>(&pl)) return r;
        std::memcpy(ss.key, key, sizeof key);
        ss.tables_valid = true;
    }
    Batch bt;
    bt.nch = 1; bt.counts = &n_vis; bt.freqs = &freq_hz; bt.total = n_vis; bt.max_count = n_vis;
    if (!(freq_hz > 0.0) || !std::isfinite(freq_hz)) return fail(WSIMG_E_INVALID, "freq_hz must be finite and > 0");
    WS_HIP(hipSetDevice(pl.device));
    wsimg_status r = f32 ? run_image<float>(&pl, bt, uvw, vis, wts, image_out, false)
                         : run_image<double>(&pl, bt, uvw, vis, wts, image_out, false);
    if (r) return r;
    return finish_call(&pl, 1, stats);
}

}  // namespace

extern "C" {

int32_t wsimg_version(void) { return 1; }

const char* wsimg_status_string(wsimg_status s) {
    switch (s) {
        case WSIMG_OK: return "ok";
        case WSIMG_E_INVALID: return "invalid argument";
        case WSIMG_E_NOMEM: return "out of memory";
        case WSIMG_E_HIP: return "HIP runtime error";
        case WSIMG_E_EMPTY: return "zero total weight after drops";
        case WSIMG_E_CAPACITY: return "more visibilities than the plan's max_vis";
        case WSIMG_E_UNSUPPORTED: return "unsupported parameters";
    }
    return "unknown status";
}

const char* wsimg_last_error(void) { return g_last_error.c_str(); }

const char* wsimg_stage_name(int32_t stage) {
    return (stage >= 0 && stage < WSIMG_N_KERNELS) ? kStageNames[stage] : nullptr;
}

wsimg_status wsimg_plan_create(wsimg_plan** out, const wsimg_params* p, int64_t max_vis, void* hip_stream) {
    return create(out, p, max_vis, 1, hip_stream);
}

wsimg_status wsimg_plan_create_batch(wsimg_plan** out, const wsimg_params* p, int64_t max_vis,
                                     int32_t max_channels, void* hip_stream) {
    return create(out, p, max_vis, max_channels, hip_stream);
}

wsimg_status wsimg_plan_destroy(wsimg_plan* plan) {
    if (!plan) return WSIMG_OK;
    (void)hipSetDevice(plan->device);
    (void)hipStreamSynchronize(plan->stream);
    release(plan);
    delete plan;
    return WSIMG_OK;
}

wsimg_status wsimg_plan_set_stream(wsimg_plan* plan, void* hip_stream) {
    if (!plan) return fail(WSIMG_E_INVALID, "plan is NULL");
    plan->stream = (hipStream_t)hip_stream;
    return WSIMG_OK;
}

wsimg_status wsimg_plan_get_info(const wsimg_plan* plan, wsimg_plan_info* info) {
    if (!plan || !info) return fail(WSIMG_E_INVALID, "plan or info is NULL");
    fill_info(plan, info);
    return WSIMG_OK;
}

wsimg_status wsimg_plan_query(const wsimg_params* p, int64_t max_vis, int32_t max_channels, wsimg_plan_info* info) {
    if (!info) return fail(WSIMG_E_INVALID, "info is NULL");
    wsimg_plan q;
    if (auto r = plan_geometry(&q, p, max_vis, max_channels)) return r;
    int64_t bytes = 0;
    for_each_allocation(&q, [&bytes](void**, size_t b, const char*) {
        bytes += (int64_t)(b == 0 ? 256 : b);
        return WSIMG_OK;
    });
    q.device_bytes = bytes;
    fill_info(&q, info);
    return WSIMG_OK;
}

wsimg_status wsimg_image(wsimg_plan* plan, int64_t n_vis, const double* uvw_m, const void* vis,
                         const void* weights, double freq_hz, void* image_out, wsimg_stats* stats) {
    return dispatch(plan, 1, &n_vis, uvw_m, vis, weights, &freq_hz, image_out, stats, false);
}

wsimg_status wsimg_image_batch(wsimg_plan* plan, int32_t n_channels, const int64_t* row_counts,
                               const double* uvw_m, const void* vis, const void* weights,
                               const double* freqs_hz, void* images_out, wsimg_stats* stats) {
    return dispatch(plan, n_channels, row_counts, uvw_m, vis, weights, freqs_hz, images_out, stats, false);
}

wsimg_status wsimg_predict(wsimg_plan* plan, int64_t n_vis, const double* uvw_m, const void* weights,
                           double freq_hz, const void* image_in, void* vis_out, wsimg_stats* stats) {
    return dispatch_predict(plan, n_vis, uvw_m, weights, freq_hz, image_in, vis_out, stats);
}

wsimg_status wsimg_grid(wsimg_plan* plan, int64_t n_vis, const double* uvw_m, const void* vis,
                        const void* weights, double freq_hz, void* grid_out, wsimg_stats* stats) {
    return dispatch(plan, 1, &n_vis, uvw_m, vis, weights, &freq_hz, grid_out, stats, true);
}

wsimg_status wsimg_image_noalloc(const wsimg_params* p, int64_t n_vis, const double* uvw_m, const void* vis,
                                 const void* weights, double freq_hz, void* image_out, void* hip_stream,
                                 wsimg_stats* stats) {
    return image_noalloc(p, n_vis, uvw_m, vis, weights, freq_hz, image_out, hip_stream, stats);
}

wsimg_status wsimg_set_timing(wsimg_plan* plan, int32_t enable) {
    if (!plan) return fail(WSIMG_E_INVALID, "plan is NULL");
    WS_HIP(hipStreamSynchronize(plan->stream));
    for (auto& e : plan->pending) plan->spare.push_back(e);
    plan->pending.clear();
    plan->totals = wsimg_timing{};
    plan->timing = enable != 0;
    return WSIMG_OK;
}

wsimg_status wsimg_read_timing(wsimg_plan* plan, wsimg_timing* out) {
    if (!plan || !out) return fail(WSIMG_E_INVALID, "plan or out is NULL");
    WS_HIP(hipStreamSynchronize(plan->stream));
    for (auto& ev : plan->pending) {
        for (int k = 0; k < WSIMG_N_KERNELS; ++k) {
            float ms = 0.f;
            WS_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            plan->totals.ms[k] += ms;
        }
        float tot = 0.f;
        WS_HIP(hipEventElapsedTime(&tot, ev[0], ev[WSIMG_N_KERNELS]));
        plan->totals.ms_total += tot;
        plan->totals.calls += 1;
        plan->spare.push_back(ev);
    }
    plan->pending.clear();
    *out = plan->totals;
    return WSIMG_OK;
}

}  // extern "C"
