// C ABI of the w-stacking imager: plan set-up, argument checks, launches.
// The declarations and their contracts are in include/wsimg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
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
                                            "scatter", "grid_rows", "cols_stack"};

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }

}  // namespace

struct wsimg_plan {
    wsimg_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t max_vis = 0;
    Geom g{};
    int nt1 = 0, nt2 = 0;          // threads of the gridding and stacking work-groups
    size_t lds1 = 0, lds2 = 0;     // their dynamic LDS bytes
    int64_t nb = 0;                // buckets
    size_t cbytes = 0, rbytes = 0; // complex / real element bytes
    int nparts = 1024;             // reduction partials
    // device memory
    Partial* partials = nullptr;
    Scalars* scalars = nullptr;
    uint32_t *counts = nullptr, *offsets = nullptr, *tile_sums = nullptr;
    uint8_t *occ = nullptr, *plane_occ = nullptr;
    uint32_t* list = nullptr;      // work list of occupied strips
    int persist_blocks = 256;      // work-groups of the persistent gridding kernel
    uint32_t *key = nullptr, *rank = nullptr, *rec_cell = nullptr;
    void *rec = nullptr, *inter = nullptr;
    void *tw = nullptr, *inv_taper = nullptr, *kbc = nullptr;
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

void release(wsimg_plan* pl) {
    for (void* a : pl->allocations) (void)hipFree(a);
    pl->allocations.clear();
    for (auto& ev : pl->pending) for (auto e : ev) (void)hipEventDestroy(e);
    for (auto& ev : pl->spare) for (auto e : ev) (void)hipEventDestroy(e);
    pl->pending.clear();
    pl->spare.clear();
}

wsimg_status validate_params(const wsimg_params* p, int64_t max_vis) {
    if (!p) return fail(WSIMG_E_INVALID, "params is NULL");
    if (p->precision != WSIMG_F32 && p->precision != WSIMG_F64)
        return fail(WSIMG_E_INVALID, "precision must be WSIMG_F32 or WSIMG_F64");
    if (!is_pow2(p->n) || p->n < 16 || p->n > 16384)
        return fail(WSIMG_E_INVALID, "n must be a power of two in [16, 16384]");
    if (p->n > 8192)
        return fail(WSIMG_E_UNSUPPORTED, "this build images n <= 8192");
    if (p->n_wplanes < 1 || p->n_wplanes > 4096)
        return fail(WSIMG_E_INVALID, "n_wplanes must be in [1, 4096]");
    if (p->support < 3 || p->support > kMaxSupport || (p->support & 1) == 0 || p->support >= p->n)
        return fail(WSIMG_E_INVALID, "support must be odd, in [3, 15] and below n");
    if (!(p->pixel_rad > 0.0) || !std::isfinite(p->pixel_rad))
        return fail(WSIMG_E_INVALID, "pixel_rad must be finite and > 0");
    const double lmax = 0.5 * p->n * p->pixel_rad;
    if (!(2.0 * lmax * lmax < 1.0))
        return fail(WSIMG_E_INVALID, "field too wide: a corner pixel has l^2 + m^2 >= 1");
    if (!std::isfinite(p->beta)) return fail(WSIMG_E_INVALID, "beta must be finite");
    if (p->reserved != 0 || (p->flags & ~WSIMG_FIXED_WRANGE) != 0)
        return fail(WSIMG_E_INVALID, "unknown flags or reserved field set");
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
    const int n = pl->p.n, W = pl->p.support;
    const host::ld beta = (host::ld)pl->p.beta;
    const int deg = KbDeg<R>::value;
    std::vector<host::ld> coef = host::kb_tap_polynomials(W, beta, deg);
    std::vector<R> hc(coef.size());
    for (size_t i = 0; i < coef.size(); ++i) hc[i] = (R)coef[i];
    std::vector<host::ld> taper = host::inverse_taper(n, W, beta);
    std::vector<R> ht(n);
    for (int i = 0; i < n; ++i) ht[i] = (R)taper[i];
    std::vector<host::ld> tre, tim;
    host::twiddles(n, tre, tim);
    std::vector<C> htw(n);
    for (int i = 0; i < n; ++i) { htw[i].x = (R)tre[i]; htw[i].y = (R)tim[i]; }
    WS_HIP(hipMemcpy(pl->kbc, hc.data(), hc.size() * sizeof(R), hipMemcpyHostToDevice));
    WS_HIP(hipMemcpy(pl->inv_taper, ht.data(), ht.size() * sizeof(R), hipMemcpyHostToDevice));
    WS_HIP(hipMemcpy(pl->tw, htw.data(), htw.size() * sizeof(C), hipMemcpyHostToDevice));
    return WSIMG_OK;
}

// Fix the work-group shapes of a (precision, n) plan and raise the dynamic-LDS limits.
template <typename R, int LOG2N>
wsimg_status configure_shape(wsimg_plan* pl) {
    using SH = Shape<R, LOG2N>;
    Geom& g = pl->g;
    g.H = SH::H; g.log2H = Log2Of<SH::H>::value_any; g.S = SH::N / SH::H;
    g.B = SH::B; g.log2B = Log2Of<SH::B>::value_any; g.NB = SH::N / SH::B;
    pl->nt1 = SH::NT1;
    pl->nt2 = SH::NT2;
    pl->lds1 = SH::LDS1_BYTES;
    pl->lds2 = SH::LDS2_BYTES;
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_rows<R, LOG2N>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_grid_only<R, LOG2N>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds1));
    WS_HIP(hipFuncSetAttribute((const void*)k_cols_stack<R, LOG2N>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->lds2));
    return WSIMG_OK;
}

#define WS_LAUNCH_CHECK(what)                                                               \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess) return fail(WSIMG_E_HIP, std::string("launch ") + what + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename R, int LOG2N>
wsimg_status launch_grid_rows(wsimg_plan* pl, bool fft, void* out) {
    using C = typename Cx<R>::T;
    const Geom g = pl->g;
    if (fft) {
        hipLaunchKernelGGL((k_grid_rows<R, LOG2N>), dim3((unsigned)pl->persist_blocks), dim3(pl->nt1), pl->lds1,
                           pl->stream, g, (int)pl->nb, pl->scalars, pl->list, pl->offsets, pl->rec_cell,
                           (const void*)pl->rec, (const R*)pl->kbc, (const C*)pl->tw,
                           (C*)out);
    } else {
        hipLaunchKernelGGL((k_grid_only<R, LOG2N>), dim3((unsigned)(g.nw * g.S)), dim3(pl->nt1), pl->lds1,
                           pl->stream, g, pl->offsets, pl->occ, pl->rec_cell, (const void*)pl->rec,
                           (const R*)pl->kbc, (C*)out);
    }
    WS_LAUNCH_CHECK("grid_rows");
    return WSIMG_OK;
}

template <typename R, int LOG2N>
wsimg_status launch_cols(wsimg_plan* pl, void* image) {
    using C = typename Cx<R>::T;
    const Geom g = pl->g;
    hipLaunchKernelGGL((k_cols_stack<R, LOG2N>), dim3((unsigned)g.NB), dim3(pl->nt2), pl->lds2, pl->stream, g,
                       pl->scalars, pl->occ, pl->plane_occ, (const C*)pl->inter, (const C*)pl->tw,
                       (const R*)pl->inv_taper, (R*)image);
    WS_LAUNCH_CHECK("cols_stack");
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

template <typename R> wsimg_status configure(wsimg_plan* pl) { WS_SIZE_DISPATCH(R, pl->g.log2n, configure_shape, pl) }
template <typename R> wsimg_status grid_rows(wsimg_plan* pl, bool fft, void* out) {
    WS_SIZE_DISPATCH(R, pl->g.log2n, launch_grid_rows, pl, fft, out)
}
template <typename R> wsimg_status cols_stack(wsimg_plan* pl, void* image) {
    WS_SIZE_DISPATCH(R, pl->g.log2n, launch_cols, pl, image)
}

wsimg_status validate_call(wsimg_plan* pl, int64_t n_vis, const double* uvw, const void* vis,
                           const void* weights, double freq_hz, void* out) {
    if (!pl) return fail(WSIMG_E_INVALID, "plan is NULL");
    if (n_vis < 0) return fail(WSIMG_E_INVALID, "n_vis < 0");
    if (n_vis > pl->max_vis) return fail(WSIMG_E_CAPACITY, "n_vis exceeds the plan's max_vis");
    if (n_vis > 0 && (!uvw || !vis || !weights)) return fail(WSIMG_E_INVALID, "input pointer is NULL");
    if (!out) return fail(WSIMG_E_INVALID, "output pointer is NULL");
    if (!(freq_hz > 0.0) || !std::isfinite(freq_hz)) return fail(WSIMG_E_INVALID, "freq_hz must be finite and > 0");
    return WSIMG_OK;
}

struct Stamp {
    wsimg_plan* pl;
    std::array<hipEvent_t, WSIMG_N_KERNELS + 1>* ev = nullptr;
    explicit Stamp(wsimg_plan* p) : pl(p) {}
    wsimg_status begin() {
        if (!pl->timing) return WSIMG_OK;
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

inline unsigned blocks_for(int64_t count, int threads) {
    return (unsigned)((count + threads - 1) / threads);
}

// Stages shared by wsimg_image and wsimg_grid: counters, plane range, bucket sort.
template <typename R>
wsimg_status run_sort(wsimg_plan* pl, Stamp& st, int64_t M, const double* uvw, const void* vis,
                      const void* wts, double freq) {
    using C = typename Cx<R>::T;
    const Geom g = pl->g;
    hipStream_t s = pl->stream;
    const int64_t nbk = pl->nb;
    const int64_t ncnt = nbk * kReplicas;
    hipLaunchKernelGGL(k_fill_u32, dim3(std::min<int64_t>(blocks_for(ncnt, 256), 8192)), dim3(256), 0, s,
                       pl->counts, ncnt, 0u);
    WS_LAUNCH_CHECK("fill");
    if (auto r = st.after(0)) return r;

    const int64_t chunk = std::max<int64_t>(1, (M + pl->nparts - 1) / pl->nparts);
    const int nparts = M > 0 ? (int)((M + chunk - 1) / chunk) : 0;
    if (nparts > 0) {
        hipLaunchKernelGGL((k_reduce<R>), dim3(nparts), dim3(256), 0, s, M, chunk, uvw,
                           (const R*)wts, freq, g, pl->partials);
        WS_LAUNCH_CHECK("reduce");
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, nparts, pl->partials, g, M, pl->scalars);
    WS_LAUNCH_CHECK("finalize");
    if (auto r = st.after(1)) return r;

    if (M > 0) {
        hipLaunchKernelGGL((k_key<R>), dim3(blocks_for(M, 256)), dim3(256), 0, s, M, uvw, (const R*)wts,
                           freq, g, pl->scalars, pl->key, pl->rank, pl->counts);
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
    hipLaunchKernelGGL(k_occupancy, dim3(blocks_for(nbk, 256)), dim3(256), 0, s, (int)nbk, pl->offsets, g,
                       pl->occ, pl->plane_occ, pl->list, pl->scalars);
    WS_LAUNCH_CHECK("occupancy");
    if (auto r = st.after(3)) return r;

    if (M > 0) {
        hipLaunchKernelGGL((k_scatter<R, R>), dim3(blocks_for(M, 256)), dim3(256), 0, s, M, uvw,
                           (const C*)vis, (const R*)wts, freq, g, pl->key, pl->rank, pl->offsets,
                           pl->rec_cell, pl->rec);
        WS_LAUNCH_CHECK("scatter");
    }
    if (auto r = st.after(4)) return r;
    return WSIMG_OK;
}

template <typename R>
wsimg_status run_image(wsimg_plan* pl, int64_t M, const double* uvw, const void* vis, const void* wts,
                       double freq, void* image, bool grid_only) {
    Stamp st(pl);
    if (auto r = st.begin()) return r;
    if (auto r = run_sort<R>(pl, st, M, uvw, vis, wts, freq)) return r;
    if (grid_only) {
        if (auto r = grid_rows<R>(pl, false, image)) return r;
        if (auto r = st.after(5)) return r;
        if (auto r = st.after(6)) return r;
        return WSIMG_OK;
    }
    if (auto r = grid_rows<R>(pl, true, pl->inter)) return r;
    if (auto r = st.after(5)) return r;
    if (auto r = cols_stack<R>(pl, image)) return r;
    if (auto r = st.after(6)) return r;
    return WSIMG_OK;
}

wsimg_status finish_call(wsimg_plan* pl, wsimg_stats* stats) {
    if (!stats) return WSIMG_OK;
    Scalars h{};
    WS_HIP(hipMemcpyAsync(&h, pl->scalars, sizeof h, hipMemcpyDeviceToHost, pl->stream));
    WS_HIP(hipStreamSynchronize(pl->stream));
    stats->n_in = (int64_t)h.n_in;
    stats->n_gridded = (int64_t)h.n_kept;
    stats->n_dropped = (int64_t)(h.n_in - h.n_kept);
    stats->sum_w = h.sum_w;
    stats->w_lo = h.w_lo;
    stats->w_hi = h.w_hi;
    stats->n_strips_occupied = (int64_t)h.n_occ;
    stats->n_planes_occupied = (int64_t)h.n_planes;
    if (!(h.sum_w != 0.0)) return fail(WSIMG_E_EMPTY, "the kept visibilities have zero total weight");
    return WSIMG_OK;
}

wsimg_status dispatch(wsimg_plan* pl, int64_t n_vis, const double* uvw, const void* vis, const void* wts,
                      double freq, void* out, wsimg_stats* stats, bool grid_only) {
    if (auto r = validate_call(pl, n_vis, uvw, vis, wts, freq, out)) return r;
    WS_HIP(hipSetDevice(pl->device));
    wsimg_status r = pl->p.precision == WSIMG_F32
                         ? run_image<float>(pl, n_vis, uvw, vis, wts, freq, out, grid_only)
                         : run_image<double>(pl, n_vis, uvw, vis, wts, freq, out, grid_only);
    if (r) return r;
    return finish_call(pl, stats);
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
    if (!out) return fail(WSIMG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (auto r = validate_params(p, max_vis)) return r;

    wsimg_plan* pl = new (std::nothrow) wsimg_plan();
    if (!pl) return fail(WSIMG_E_NOMEM, "host allocation of the plan failed");
    pl->p = *p;
    if (!(pl->p.beta > 0.0)) pl->p.beta = 2.34 * pl->p.support;
    pl->max_vis = max_vis;
    pl->stream = (hipStream_t)hip_stream;

    const bool f32 = p->precision == WSIMG_F32;
    pl->rbytes = f32 ? 4 : 8;
    pl->cbytes = 2 * pl->rbytes;
    const int n = p->n;
    Geom& g = pl->g;
    g.n = n; g.log2n = ilog2(n); g.nw = p->n_wplanes; g.support = p->support; g.half = (p->support - 1) / 2;
    g.du = 1.0 / ((double)n * p->pixel_rad);
    g.half_n = (double)n / 2.0;
    g.pixel = p->pixel_rad;
    g.fixed_range = (p->flags & WSIMG_FIXED_WRANGE) ? 1 : 0;
    g.w_lo_fixed = p->w_lo; g.w_hi_fixed = p->w_hi;
    {
        wsimg_status rs = f32 ? configure<float>(pl) : configure<double>(pl);
        if (rs) { delete pl; return rs; }
    }
    pl->nb = (int64_t)g.nw * g.S;

    hipError_t he = hipGetDevice(&pl->device);
    if (he != hipSuccess) { delete pl; return fail(WSIMG_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he)); }
    int cus = 0;
    he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device);
    if (he != hipSuccess || cus <= 0) { delete pl; return fail(WSIMG_E_HIP, "hipDeviceGetAttribute(CU count) failed"); }
    // as many strip work-groups as fit at once: one per CU while the LDS strip exceeds 80 KB
    pl->persist_blocks = cus * std::max(1, (int)((160 * 1024) / std::max<size_t>(pl->lds1, 1)));

    wsimg_status r = WSIMG_OK;
    const size_t mv = (size_t)std::max<int64_t>(max_vis, 1);
    const size_t cells = (size_t)g.nw * (size_t)n * (size_t)n;
    void* tmp = nullptr;
#define ALLOC(field, bytes, name)                                                  \
    if (!r) { r = dev_alloc(pl, &tmp, (bytes), name); pl->field = (decltype(pl->field))tmp; }
    ALLOC(partials, sizeof(Partial) * pl->nparts, "partials");
    ALLOC(scalars, sizeof(Scalars), "scalars");
    ALLOC(counts, sizeof(uint32_t) * pl->nb * kReplicas, "counts");
    ALLOC(offsets, sizeof(uint32_t) * (pl->nb * kReplicas + 1), "offsets");
    ALLOC(tile_sums, sizeof(uint32_t) * ((pl->nb * kReplicas + kScanTile - 1) / kScanTile), "scan tiles");
    ALLOC(occ, (size_t)pl->nb, "occupancy");
    ALLOC(list, sizeof(uint32_t) * (size_t)pl->nb, "strip work list");
    ALLOC(plane_occ, (size_t)g.nw, "plane occupancy");
    ALLOC(key, sizeof(uint32_t) * mv, "keys");
    ALLOC(rank, sizeof(uint32_t) * mv, "ranks");
    ALLOC(rec_cell, f32 ? 256 : sizeof(uint32_t) * mv, "record cells");
    ALLOC(rec, (f32 ? 16 : 32) * mv, "records");
    ALLOC(inter, pl->cbytes * cells, "row-transformed planes");
    ALLOC(tw, pl->cbytes * n, "twiddles");
    ALLOC(inv_taper, pl->rbytes * n, "taper");
    ALLOC(kbc, pl->rbytes * (size_t)p->support * 17, "kernel polynomials");
#undef ALLOC
    if (!r) r = f32 ? upload_tables<float>(pl) : upload_tables<double>(pl);
    if (r) { release(pl); delete pl; return r; }
    *out = pl;
    return WSIMG_OK;
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
    info->n = plan->p.n;
    info->n_wplanes = plan->p.n_wplanes;
    info->support = plan->p.support;
    info->precision = plan->p.precision;
    info->strip_rows = plan->g.H;
    info->col_block = plan->g.B;
    info->n_buckets = plan->nb;
    info->max_vis = plan->max_vis;
    info->device_bytes = plan->device_bytes;
    return WSIMG_OK;
}

wsimg_status wsimg_image(wsimg_plan* plan, int64_t n_vis, const double* uvw_m, const void* vis,
                         const void* weights, double freq_hz, void* image_out, wsimg_stats* stats) {
    return dispatch(plan, n_vis, uvw_m, vis, weights, freq_hz, image_out, stats, false);
}

wsimg_status wsimg_grid(wsimg_plan* plan, int64_t n_vis, const double* uvw_m, const void* vis,
                        const void* weights, double freq_hz, void* grid_out, wsimg_stats* stats) {
    return dispatch(plan, n_vis, uvw_m, vis, weights, freq_hz, grid_out, stats, true);
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
