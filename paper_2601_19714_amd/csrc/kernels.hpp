// The imaging kernels for gfx950.
//
//  k_fill_u32     : zero the bucket counters (a kernel, not a memset, so the stages can be
//                   captured into a graph).
//  k_reduce       : per-block partial (min w, max w, sum of weights, count) over kept rows.
//  k_finalize     : fixed-order reduction of the partials -> plane range and sum of weights.
//  k_key          : per row, the bucket (w-plane, row strip of its first tap row) and its rank
//                   inside the bucket (a counting-sort histogram, Sec. 3.2's bucket sort) on
//                   replicated counters.
//  k_scan_*       : exclusive scan of the counters (tile sums, top level, tiles).
//  k_occupancy    : strip and plane occupancy flags and counts.
//  k_scatter      : sorted records {tap origin, sub-cell offsets, W*V} (SoA).
//  k_grid_rows    : one work-group per occupied (plane, strip): Kaiser-Bessel gridding of every
//                   record whose taps reach the strip into an LDS strip (Eq. 3), then the
//                   row FFT of the strip in LDS; writes the strip in column-block layout.
//                   The FFT-less variant writes the raw grid (the gridding step alone).
//  k_cols_stack   : one work-group per block of image columns: for each plane, column FFTs
//                   in LDS, multiply by the plane's w-phase, Kahan-accumulate the real part;
//                   finally divide by the taper on both axes and the sum of weights.
//
// Every stage carries a channel index: a call images one or more channels (frequencies) at
// once.  The rows of channel c are rows [row_off[c], row_off[c+1]) of the inputs; each
// channel has its own plane range, sum of weights, buckets, intermediate and image.  Row
// kernels run on a grid whose y index is the channel; the gridding work list spans all
// channels.
#pragma once

#include "device_common.hpp"
#include "fft_lds.hpp"

namespace wsimg {

// Plan constants handed to every kernel by value.
// n is the grid side: the image side n_img times the padding (1 or 2); the image is the grid
// image's central n_img x n_img, starting at row and column crop = (n - n_img) / 2.
struct Geom {
    int n, log2n, nw, support, half;
    int n_img, crop;
    size_t plane_elems;     // elements of one plane of the intermediate: n * n_img
    int H, log2H, S;        // grid rows per strip, strips per plane
    int nb1;                // buckets per channel: nw * S
    int B, log2B, NB;       // columns per layout block of the intermediate; prediction column blocks
    int fixed_range;
    int unnormalized;       // the image is not divided by the sum of weights
    int fold_w;             // w-folding (rows with w < 0 as their conjugate partners)
    int wsup, whalf;        // w-kernel across planes: support Ww (0: nearest plane) and (Ww - 1) / 2
    double du, half_n, pixel;
    double w_lo_fixed, w_hi_fixed;
    double wbeta, wscale;   // the w-kernel's shape and Ww / I0(beta_w)
};

// Per-call channel table (device arrays).
struct Chan {
    const int64_t* row_off;   // [nch + 1]: rows of channel c are [row_off[c], row_off[c + 1])
    const double* freq;       // [nch], Hz
};

// Per channel, written by k_finalize (and k_occupancy's counts), read by the later stages.
struct Scalars {
    double w_lo, w_hi, dw, sum_w;
    unsigned long long n_kept, n_in, n_occ, n_planes;
    double w_c0;            // the w-kernel's plane 0 centre, w_lo - h dw (planes at w_c0 + k dw)
};

// The gridding work list of occupied strips of all channels: heavy ones from the front,
// light ones from the back; next is the persistent kernel's fetch counter, n_split the number
// of strips split into parts (below).
// Each fetch counter has a 128-byte line of its own: the eight per-XCD counters on one line
// made the atomics of the whole grid queue on it (64 channels of 1024^2: gridding 6.2 ms against
// 4.4 ms with a line each; 8192^2: 16.9 against 16.4 ms).
struct WorkList {
    unsigned int n_heavy, n_light, n_split, pad0[29];
    unsigned int next, pad1[31];
    struct { unsigned int n, pad[31]; } xnext[8];   // per-XCD counters over the light entries
    unsigned int n_big, pad2[31];                    // buckets in the big-bucket list (k_origin_sort)
};

// Heavy strips are split.  With `share` the record visits of the call over the gridding
// work-groups (each work-group's fair share, at least kMinPart), a strip of more than
// 2 * share visits would outlast the rest of the grid alone, so it is gridded as
// P = min(kMaxParts, ceil(visits / share)) parts by different work-groups (each a contiguous
// share of its records), which add their float64 strips into a global slot; the work-group
// that completes the last part takes the sum and runs the row FFT.  At most kMaxSplit strips
// per call are split (the slots' memory); the rest run whole.  A list entry's companion
// word: slot << 16 | part << 8 | parts (parts = 1: not split).
constexpr uint32_t kMinPart = 4096;
constexpr uint32_t kMaxParts = 32;
constexpr uint32_t kMaxSplit = 512;

struct Partial {
    double wmin, wmax, sumw;
    unsigned long long nk;
};

template <typename R> struct KbDeg;
template <> struct KbDeg<float> { static constexpr int value = 10; };
template <> struct KbDeg<double> { static constexpr int value = 16; };

// G(a - half - f) for f in [-1/2, 1/2]: a per-tap polynomial in f (coefficients fitted on the
// host in extended precision at Chebyshev nodes), evaluated by Horner's rule.
template <typename R>
__device__ __forceinline__ R kb_tap(const R* __restrict__ coef, int a, R f) {
    constexpr int D = KbDeg<R>::value;
    const R* c = coef + a * (D + 1);
    R acc = c[D];
#pragma unroll
    for (int d = D - 1; d >= 0; --d) acc = acc * f + c[d];
    return acc;
}

// All taps of one axis, centred: g[C + d] = G(d - f) for |d| <= h = (W - 1) / 2, C = WMAX / 2
// (tap a = h + d of the origin ⌊x + 1/2⌋ - h).  G is even, so tap h + d at offset f is tap
// h - d at offset -f: with P the polynomial of tap h - d split into its even part E(f^2) and
// odd part f O(f^2), the pair is E + f O (tap h - d) and E - f O (tap h + d), one evaluation
// of each half for two taps.
template <typename R, int WMAX>
__device__ __forceinline__ void kb_taps_centred(const R* __restrict__ coef, int h, R f, R* g) {
    constexpr int D = KbDeg<R>::value, C = WMAX / 2;
    constexpr int DE = D & ~1, DO = (D & 1) ? D : D - 1;      // highest even / odd degree
    const R f2 = f * f;
#pragma unroll
    for (int d = 0; d <= C; ++d) {
        if (d <= h) {
            const R* c = coef + (h - d) * (D + 1);
            R e = c[DE];
#pragma unroll
            for (int k = DE - 2; k >= 0; k -= 2) e = e * f2 + c[k];
            R o = c[DO];
#pragma unroll
            for (int k = DO - 2; k >= 1; k -= 2) o = o * f2 + c[k];
            const R fo = f * o;
            g[C - d] = e + fo;
            if (d > 0) g[C + d] = e - fo;
        }
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t count, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// The channel table of a one-channel call, written on the device from kernel arguments (the
// allocation-free entry point has no pinned staging buffer).
__global__ void k_set_channel(int64_t* __restrict__ row_off, double* __restrict__ freq, int64_t n_vis,
                              double freq_hz) {
    if (threadIdx.x == 0) {
        row_off[0] = 0;
        row_off[1] = n_vis;
        freq[0] = freq_hz;
    }
}

template <typename T>
__device__ __forceinline__ T wave_reduce_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_reduce_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_reduce_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block (b, c) of 256 threads covers rows [b*chunk, min(count_c, (b+1)*chunk)) of channel c.
template <typename WT>
__global__ void __launch_bounds__(256)
k_reduce(Chan ch, int64_t chunk, int nparts, const double* __restrict__ uvw, const WT* __restrict__ wts,
         Geom g, Partial* __restrict__ part) {
    const int c = blockIdx.y;
    const int64_t r1 = ch.row_off[c + 1];
    const int64_t beg = ch.row_off[c] + blockIdx.x * chunk;
    const int64_t end = beg + chunk < r1 ? beg + chunk : r1;
    const double freq = ch.freq[c];
    double wmin = INFINITY, wmax = -INFINITY, sw = 0.0;
    unsigned long long nk = 0;
    for (int64_t m = beg + threadIdx.x; m < end; m += blockDim.x) {
        const double wt = (double)wts[m];
        RowGeom rg = row_geometry(uvw, m, freq, g.du, g.half_n, wt, g.n, g.support, g.fold_w);
        if (rg.keep) {
            sw += wt;
            nk += 1;
            if (wt > 0.0) { wmin = fmin(wmin, rg.w); wmax = fmax(wmax, rg.w); }
        }
    }
    sw = wave_reduce_sum(sw);
    nk = wave_reduce_sum(nk);
    wmin = wave_reduce_min(wmin);
    wmax = wave_reduce_max(wmax);
    __shared__ Partial sh[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = Partial{wmin, wmax, sw, nk};
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial t = sh[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            t.wmin = fmin(t.wmin, sh[i].wmin);
            t.wmax = fmax(t.wmax, sh[i].wmax);
            t.sumw += sh[i].sumw;
            t.nk += sh[i].nk;
        }
        part[(size_t)c * nparts + blockIdx.x] = t;
    }
}

// One block of 256 threads per channel; fixed summation order, so the sum of weights is
// reproducible.  Block 0 also resets the work list.
__global__ void __launch_bounds__(256)
k_finalize(int nparts, const Partial* __restrict__ part, Geom g, Chan ch, Scalars* __restrict__ sc,
           WorkList* __restrict__ wl) {
    __shared__ double s_sw[256], s_min[256], s_max[256];
    __shared__ unsigned long long s_nk[256];
    const int c = blockIdx.x;
    const Partial* pc = part + (size_t)c * nparts;
    double sw = 0.0, mn = INFINITY, mx = -INFINITY;
    unsigned long long nk = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        sw += pc[i].sumw; nk += pc[i].nk;
        mn = fmin(mn, pc[i].wmin); mx = fmax(mx, pc[i].wmax);
    }
    s_sw[threadIdx.x] = sw; s_min[threadIdx.x] = mn; s_max[threadIdx.x] = mx; s_nk[threadIdx.x] = nk;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_sw[threadIdx.x] += s_sw[threadIdx.x + o];
            s_nk[threadIdx.x] += s_nk[threadIdx.x + o];
            s_min[threadIdx.x] = fmin(s_min[threadIdx.x], s_min[threadIdx.x + o]);
            s_max[threadIdx.x] = fmax(s_max[threadIdx.x], s_max[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma clang fp contract(off)
        Scalars r;
        if (g.fixed_range) { r.w_lo = g.w_lo_fixed; r.w_hi = g.w_hi_fixed; }
        else if (s_min[0] <= s_max[0]) { r.w_lo = s_min[0]; r.w_hi = s_max[0]; }
        else { r.w_lo = 0.0; r.w_hi = 0.0; }
        if (g.wsup) {       // Ww taps of every row on the planes: Nw - Ww plane spacings
            r.dw = (r.w_hi - r.w_lo) / (double)(g.nw - g.wsup);
            r.w_c0 = r.w_lo - (double)g.whalf * r.dw;
        } else {
            r.dw = (r.w_hi - r.w_lo) / (double)g.nw;
            r.w_c0 = r.w_lo + 0.5 * r.dw;
        }
        r.sum_w = s_sw[0];
        r.n_kept = s_nk[0];
        r.n_in = (unsigned long long)(ch.row_off[c + 1] - ch.row_off[c]);
        r.n_occ = 0;
        r.n_planes = 0;
        sc[c] = r;
        if (c == 0) {       // the counters only (a whole-struct store takes 25 us from one thread)
            wl->n_heavy = 0u;
            wl->n_light = 0u;
            wl->n_split = 0u;
            wl->next = 0u;
#pragma unroll
            for (int x = 0; x < 8; ++x) wl->xnext[x].n = 0u;
            wl->n_big = 0u;
        }
    }
}

// Bucket counters are replicated kReplicas times, laid out [bucket][replica]; the rows of
// row block b of a channel (kKeyRows rows) count in replica b mod kReplicas.  The rows of one hot
// bucket (tens of thousands near the uv-plane centre) then spread their atomics over
// kReplicas addresses instead of one, and the bucket's rows still end up contiguous after
// the scan.  (Blocks of consecutive rows, not single rows: a bucket's records keep their
// time-major order, so the lanes of a gridding wave hold different baselines and rarely hit
// the same cell.)  Bucket id: channel * nb1 + plane * S + strip.
constexpr int kReplicas = 64;
constexpr int kLogReplicas = 6;

// Ranks inside a (bucket, replica) counter: the block's rows group their keys in an LDS hash
// table; one global atomic per distinct key of the block, and each row's rank is that atomic's
// return plus its order in the table slot (one atomic per row serialises the lanes that hit a
// hot bucket; a per-wave leader loop was slower on many small channels).
// A block of kKeyThreads threads takes kKeyRowsPerThread rows each: consecutive rows (one time
// step's baselines, then the next steps') repeat keys more often over a longer span (the 4096^2
// MeerKAT-shaped set: 0.77 distinct keys per row over 256 rows, 0.51 over 1024), so a longer block takes fewer global
// atomics, and fewer of them meet on one counter.  On the 8192^2 LOFAR-shaped image (where
// almost every row of one time step has a bucket of its own) the key stage took 2.26 ms with
// 1024-row blocks, 0.92 ms with 4096 (about two time steps of the 60-station array) and 0.59 ms
// with 8192; at 4096^2 0.19, 0.10 and 0.076 ms.
#ifndef WSIMG_KEY_THREADS
#define WSIMG_KEY_THREADS 1024
#endif
#ifndef WSIMG_KEY_ROWS_PER_THREAD
#define WSIMG_KEY_ROWS_PER_THREAD 8
#endif
constexpr int kKeyThreads = WSIMG_KEY_THREADS;
constexpr int kKeyRowsPerThread = WSIMG_KEY_ROWS_PER_THREAD;
constexpr int kKeyRows = kKeyThreads * kKeyRowsPerThread;
static_assert(kKeyThreads == 256 || kKeyThreads == 512 || kKeyThreads == 1024, "k_key block size");
static_assert(kKeyRowsPerThread >= 1 && kKeyRowsPerThread <= 8, "k_key rows per thread");
// slots of the block's hash table (more than the block's rows, so a free slot always exists);
// two 4-byte words each, in dynamic LDS.  1.25 slots per row keep the table at 80 KB for 8192
// rows, two blocks per CU (the distinct keys of a block are about a quarter of its rows, so
// probes stay short); 2 per row (128 KB, one block per CU) made the 8192^2 key stage 0.87 ms
// against 0.59 ms.
#ifndef WSIMG_KEY_SLOTS
#define WSIMG_KEY_SLOTS (kKeyRows + kKeyRows / 4)
#endif
constexpr int kKeySlots = WSIMG_KEY_SLOTS;
static_assert(kKeySlots > kKeyRows, "k_key hash table size");
constexpr size_t kKeyLdsBytes = (size_t)kKeySlots * 8;

// Replica of the bucket counters that row i of a channel counts in: its k_key block's index
// mod kReplicas (k_key and k_scatter must agree on it).
__device__ __forceinline__ uint32_t row_replica(int64_t i) {
    return (uint32_t)((i / kKeyRows) & (kReplicas - 1));
}

template <typename WT>
__global__ void __launch_bounds__(kKeyThreads)
k_key(Chan ch, const double* __restrict__ uvw, const WT* __restrict__ wts, Geom g,
      const Scalars* __restrict__ sc, uint32_t* __restrict__ key, uint32_t* __restrict__ rank,
      uint32_t* __restrict__ counts) {
    constexpr int KR = kKeyRowsPerThread;
    const int c = blockIdx.y;
    const int64_t r0 = ch.row_off[c], r1 = ch.row_off[c + 1];
    const int64_t b0 = r0 + (int64_t)blockIdx.x * kKeyRows;
    if (b0 >= r1) return;                                           // whole block past the channel
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    uint32_t kk[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        const int64_t m = b0 + j * kKeyThreads + threadIdx.x;
        kk[j] = kEmpty;
        if (m < r1) {
            const double wt = (double)wts[m];
            RowGeom rg = row_geometry(uvw, m, ch.freq[c], g.du, g.half_n, wt, g.n, g.support, g.fold_w);
            if (rg.keep) {
                const int k = g.wsup ? w_taps(rg.w, sc[c].w_lo, sc[c].dw, g.nw, g.whalf).k0
                                     : plane_index(rg.w, sc[c].w_lo, sc[c].dw, g.nw);
                const int p0 = (int)rg.cy - g.half;
                kk[j] = (uint32_t)(c * g.nb1 + k * g.S + (p0 >> g.log2H));
            }
        }
    }
    const uint32_t rep = row_replica((int64_t)blockIdx.x * kKeyRows);
    // block-wide aggregation through an LDS hash table (open addressing with more slots than
    // the block's rows, so a free slot always exists): each distinct key of the block takes one
    // atomic, whose return replaces the slot's count
    constexpr int kSlots = kKeySlots;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint32_t* hkey = reinterpret_cast<uint32_t*>(smem_raw);
    uint32_t* hcnt = hkey + kSlots;
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x) { hkey[i] = kEmpty; hcnt[i] = 0u; }
    __syncthreads();
    uint32_t slot[KR], local[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        slot[j] = 0;
        local[j] = 0;
        if (kk[j] != kEmpty) {
            // multiplicative hash, its high bits scaled to [0, kSlots)
            uint32_t sl = (uint32_t)(((uint64_t)(kk[j] * 2654435761u) * (uint32_t)kSlots) >> 32);
            while (true) {
                const uint32_t prev = atomicCAS(&hkey[sl], kEmpty, kk[j]);
                if (prev == kEmpty || prev == kk[j]) break;
                sl = sl + 1 == (uint32_t)kSlots ? 0u : sl + 1;
            }
            slot[j] = sl;
            local[j] = atomicAdd(&hcnt[sl], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
        const uint32_t key_i = hkey[i];
        if (key_i != kEmpty) hcnt[i] = atomicAdd(&counts[((size_t)key_i << kLogReplicas) + rep], hcnt[i]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        const int64_t m = b0 + j * kKeyThreads + threadIdx.x;
        if (m < r1) {
            key[m] = kk[j];
            rank[m] = kk[j] != kEmpty ? hcnt[slot[j]] + local[j] : 0u;
        }
    }
}

// Exclusive scan of the replicated counters (total = nb * kReplicas entries) in three
// kernels: tile sums, a one-block scan of the tile sums, then each tile's own scan.
constexpr int kScanTile = 4096;     // 256 threads x 16 entries

__global__ void __launch_bounds__(256)
k_scan_tiles(int64_t total, const uint32_t* __restrict__ counts, uint32_t* __restrict__ tile_sums) {
    __shared__ uint32_t red[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int i = 0; i < 16; ++i) {
        const int64_t e = base + (int64_t)i * 256 + threadIdx.x;
        if (e < total) s += counts[e];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = red[0];
}

// One block of 1024 threads over ntiles tile sums (in place: sums -> exclusive offsets).
__global__ void __launch_bounds__(1024)
k_scan_top(int ntiles, uint32_t* __restrict__ tile_sums) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int chunk = (ntiles + nt - 1) / nt;
    const int b0 = t * chunk;
    const int b1 = b0 + chunk < ntiles ? b0 + chunk : ntiles;
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += tile_sums[b];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {
        uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int b = b0; b < b1; ++b) { const uint32_t c = tile_sums[b]; tile_sums[b] = run; run += c; }
}

// Each thread scans 16 consecutive entries; the block scans the 256 thread totals.
__global__ void __launch_bounds__(256)
k_scan_down(int64_t total, const uint32_t* __restrict__ counts, const uint32_t* __restrict__ tile_offs,
            uint32_t* __restrict__ offsets) {
    __shared__ uint32_t part[4];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * 16;
    // a thread's 16 entries start 64-byte aligned: whole ones move as four 16-byte accesses
    const bool whole = base + 16 <= total;
    uint32_t v[16], s = 0;
    if (whole) {
        const uint4* c4 = reinterpret_cast<const uint4*>(counts + base);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 x = c4[q];
            v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = base + i < total ? counts[base + i] : 0u;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) s += v[i];
    // exclusive scan of the 256 thread sums: within each wave by shuffles, then the wave totals
    const int lane = t & 63, wave = t >> 6;
    uint32_t inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) part[wave] = inc;
    __syncthreads();
    uint32_t run = tile_offs[blockIdx.x] + (inc - s);
    for (int w = 0; w < wave; ++w) run += part[w];
    uint32_t o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) { o[i] = run; run += v[i]; }
    if (whole) {
        uint4* o4 = reinterpret_cast<uint4*>(offsets + base);
#pragma unroll
        for (int q = 0; q < 4; ++q) o4[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (base + i < total) offsets[base + i] = o[i];
    }
    if (base + 16 >= total && base < total) offsets[total] = run;   // the thread holding the last entry
}

// Strip and plane occupancy.  occ[k*S + s] = 1 when some record of plane k has a tap row
// inside strip s, i.e. one of the buckets s_lo(s)..s (the strips whose rows can reach s) is
// non-empty.  Occupied strips also go to the gridding work list: strips with more than
// kHeavyStrip record visits from the front (list[0..n_heavy)), the rest from the back
// (list[nb - n_light .. nb)), so the long ones start first.  Counts go to the scalars.
constexpr uint32_t kHeavyStrip = 4096;
// Buckets of more records than this are origin-sorted first (their list is built here): the
// uv-centre buckets of an 8192^2 image hold up to 7e5 records, each walked by one work-group,
// and started in bucket order they would begin half-way through the sort and end after it.
constexpr uint32_t kBigBucket = 16384;

__global__ void __launch_bounds__(256)
k_occupancy(int nch, const uint32_t* __restrict__ offsets, Geom g, uint8_t* __restrict__ occ,
            uint8_t* __restrict__ plane_occ, uint32_t* __restrict__ list, uint32_t* __restrict__ list_aux,
            uint32_t list_cap, uint32_t share, Scalars* __restrict__ sc, WorkList* __restrict__ wl,
            uint32_t* __restrict__ big) {
    const int total = nch * g.nb1;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t o = 0, po = 0, visits = 0;
    int c = 0;
    if (b < total) {
        // the origin sort's big buckets (bucket b itself; at most rows / kBigBucket of them)
        if (big && offsets[(size_t)(b + 1) << kLogReplicas] - offsets[(size_t)b << kLogReplicas] > kBigBucket)
            big[atomicAdd(&wl->n_big, 1u)] = (uint32_t)b;
        c = b / g.nb1;
        const int bb = b - c * g.nb1;
        const int k = bb / g.S, sidx = bb - k * g.S;
        int slo = ((sidx << g.log2H) - (g.support - 1)) >> g.log2H;
        if (slo < 0) slo = 0;
        // the planes whose rows reach plane k: k itself, or k - Ww + 1 .. k with the w-kernel
        const int klo = g.wsup ? (k - g.wsup + 1 < 0 ? 0 : k - g.wsup + 1) : k;
        for (int kk = klo; kk <= k; ++kk) {
            const int base = c * g.nb1 + kk * g.S;
            visits += offsets[(size_t)(base + sidx + 1) << kLogReplicas] - offsets[(size_t)(base + slo) << kLogReplicas];
            if (sidx == 0)
                po |= offsets[(size_t)(base + g.S) << kLogReplicas] > offsets[(size_t)base << kLogReplicas] ? 1u : 0u;
        }
        o = visits > 0 ? 1u : 0u;
        occ[b] = (uint8_t)o;
        if (sidx == 0) plane_occ[c * g.nw + k] = (uint8_t)po;
    }
    const int lane = threadIdx.x & 63;
    const unsigned long long light = __ballot(o && visits <= kHeavyStrip);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t lbase = 0;
    if (lane == 0 && light) lbase = atomicAdd(&wl->n_light, (unsigned)__popcll(light));
    lbase = __shfl(lbase, 0, 64);
    if (o && visits <= kHeavyStrip) {
        const uint32_t at = list_cap - 1 - (lbase + __popcll(light & below));
        list[at] = (uint32_t)b;
        list_aux[at] = 1u;
    } else if (o) {
        // heavy: one entry, or one per part when split (heavy strips are few: one atomic each)
        uint32_t parts = 1, slot = 0;
        if (visits > 2 * share) {
            slot = atomicAdd(&wl->n_split, 1u);
            if (slot < kMaxSplit) {
                parts = (visits + share - 1) / share;
                parts = parts > kMaxParts ? kMaxParts : parts;
            } else {
                slot = 0;
            }
        }
        const uint32_t at = atomicAdd(&wl->n_heavy, parts);
        for (uint32_t p = 0; p < parts; ++p) {
            list[at + p] = (uint32_t)b;
            list_aux[at + p] = (slot << 16) | (p << 8) | parts;
        }
    }
    // per-channel counts: one atomic per wave when the wave lies in one channel
    const int c0 = __shfl(c, 0, 64);
    if (__all(b >= total || c == c0)) {
        o = wave_reduce_sum(o);
        po = wave_reduce_sum(po);
        if (lane == 0) {
            if (o) atomicAdd(&sc[c0].n_occ, (unsigned long long)o);
            if (po) atomicAdd(&sc[c0].n_planes, (unsigned long long)po);
        }
    } else {
        if (o) atomicAdd(&sc[c].n_occ, 1ull);
        if (po) atomicAdd(&sc[c].n_planes, 1ull);
    }
}

// Sorted records.  float: one 16-byte record per row,
//   x: q0 (13 bits) | p0 mod H (5 bits) | low 14 bits of the x offset code,
//   y: high 9 bits of the x offset code | y offset code (23 bits),
//   z, w: W*V as float2,
// where an offset f = x - floor(x + 1/2) in [-1/2, 1/2) is coded as round((f + 1/2) 2^23)
// (a resolution of 1.2e-7 cells; the tap weights change by at most ~6e-8 of their peak).
// double: rec_cell (q0 | p0 << 16) plus two double2 per row: the offsets, then W*V.
constexpr double kFracScale = 8388608.0;   // 2^23

__device__ __forceinline__ uint32_t frac_code(double f) {
    int c = __double2int_rn((f + 0.5) * kFracScale);
    return (uint32_t)(c < 0 ? 0 : (c > 8388607 ? 8388607 : c));
}

// vis may be null (prediction: the records carry positions only, W*V = 0); rec_idx, when not
// null, receives each record's input row.
// rows per k_scatter block: blocks of 1024 rows (an eighth of a k_key block, whose replica they
// share) write the records of their buckets from one work-group (4096^2: 0.20 -> 0.18 ms
// against 256-row blocks, 64 channels of 1024^2 0.99 -> 0.80 ms)
#ifndef WSIMG_SCATTER_THREADS
#define WSIMG_SCATTER_THREADS 1024
#endif
constexpr int kScatterThreads = WSIMG_SCATTER_THREADS;
template <typename R, typename WT>
__global__ void __launch_bounds__(kScatterThreads)
k_scatter(Chan ch, const double* __restrict__ uvw, const typename Cx<R>::T* __restrict__ vis,
          const WT* __restrict__ wts, Geom g, const uint32_t* __restrict__ key,
          const uint32_t* __restrict__ rank, const uint32_t* __restrict__ offsets,
          uint32_t* __restrict__ rec_cell, void* __restrict__ rec, uint32_t* __restrict__ rec_idx,
          const Scalars* __restrict__ sc, R* __restrict__ rec_w) {
    using C = typename Cx<R>::T;
    const int c = blockIdx.y;
    const int64_t r0 = ch.row_off[c], r1 = ch.row_off[c + 1];
    const int64_t m = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= r1) return;
    const uint32_t kk = key[m];
    if (kk == 0xFFFFFFFFu) return;
    const double wt = (double)wts[m];
    RowGeom rg = row_geometry(uvw, m, ch.freq[c], g.du, g.half_n, wt, g.n, g.support, g.fold_w);
    const uint32_t rep = row_replica(m - r0);              // the row block's replica (as in k_key)
    const uint32_t pos = offsets[((size_t)kk << kLogReplicas) + rep] + rank[m];
    const int q0 = (int)rg.cx - g.half, p0 = (int)rg.cy - g.half;
    // a prediction's records carry no W*V: their value slot holds (1, 0) for a folded row
    C v = vis ? vis[m] : cmake<C>(rg.flip ? (R)1 : (R)0, (R)0);
    if (vis && rg.flip) v.y = -v.y;
    const R w = vis ? (R)wts[m] : (R)1;
    if (rec_idx) rec_idx[pos] = (uint32_t)m;
    if (rec_w) rec_w[pos] = (R)w_taps(rg.w, sc[c].w_lo, sc[c].dw, g.nw, g.whalf).f;   // w-kernel offset
    if constexpr (sizeof(R) == 4) {
        const uint32_t ux = frac_code(rg.x - rg.cx), uy = frac_code(rg.y - rg.cy);
        const uint32_t pr = (uint32_t)p0 & (uint32_t)(g.H - 1);
        uint4 q;
        q.x = (uint32_t)q0 | (pr << 13) | ((ux & 0x3FFFu) << 18);
        q.y = (ux >> 14) | (uy << 9);
        q.z = __float_as_uint(w * v.x);
        q.w = __float_as_uint(w * v.y);
        reinterpret_cast<uint4*>(rec)[pos] = q;
    } else {
        rec_cell[pos] = (uint32_t)q0 | ((uint32_t)p0 << 16);
        double2* r2 = reinterpret_cast<double2*>(rec);
        r2[2 * (size_t)pos] = make_double2(rg.x - rg.cx, rg.y - rg.cy);
        r2[2 * (size_t)pos + 1] = make_double2(w * v.x, w * v.y);
    }
}

// One record as stored.
template <typename R> struct RawRec;
template <> struct RawRec<float> { uint4 q; };
template <> struct RawRec<double> { uint32_t cell; double2 f, v; };

template <typename R>
__device__ __forceinline__ RawRec<R> fetch_record(const uint32_t* __restrict__ rec_cell,
                                                  const void* __restrict__ rec, uint32_t r) {
    RawRec<R> x;
    if constexpr (sizeof(R) == 4) {
        x.q = reinterpret_cast<const uint4*>(rec)[r];
    } else {
        x.cell = rec_cell[r];
        const double2* r2 = reinterpret_cast<const double2*>(rec);
        x.f = r2[2 * (size_t)r];
        x.v = r2[2 * (size_t)r + 1];
    }
    return x;
}

template <typename R>
__device__ __forceinline__ void store_record(uint32_t* __restrict__ rec_cell, void* __restrict__ rec,
                                             uint32_t r, const RawRec<R>& x) {
    if constexpr (sizeof(R) == 4) {
        reinterpret_cast<uint4*>(rec)[r] = x.q;
    } else {
        rec_cell[r] = x.cell;
        double2* r2 = reinterpret_cast<double2*>(rec);
        r2[2 * (size_t)r] = x.f;
        r2[2 * (size_t)r + 1] = x.v;
    }
}

// Tap origin (q0, p0), sub-cell offsets and W*V in the plan precision; strip is the strip of
// the record's bucket (the float record keeps only p0 mod H).
template <typename R>
__device__ __forceinline__ void decode_record(const RawRec<R>& x, int strip, int log2H, int& q0, int& p0,
                                              typename Cx<R>::T& fr, typename Cx<R>::T& v) {
    using C = typename Cx<R>::T;
    if constexpr (sizeof(R) == 4) {
        const uint4 q = x.q;
        q0 = (int)(q.x & 0x1FFFu);
        p0 = (strip << log2H) + (int)((q.x >> 13) & 0x1Fu);
        const uint32_t ux = (q.x >> 18) | ((q.y & 0x1FFu) << 14), uy = q.y >> 9;
        const float inv = 1.0f / 8388608.0f;
        fr = cmake<C>((float)ux * inv - 0.5f, (float)uy * inv - 0.5f);
        v = cmake<C>(__uint_as_float(q.z), __uint_as_float(q.w));
    } else {
        q0 = (int)(x.cell & 0xFFFFu);
        p0 = (int)(x.cell >> 16);
        fr = x.f;
        v = x.v;
    }
}

// A lane's record (or value) from lane src of the wave.
template <typename R> __device__ __forceinline__ R shfl_real(R v, int src) { return __shfl(v, src, 64); }
template <typename R> __device__ __forceinline__ RawRec<R> shfl_record(const RawRec<R>& x, int src) {
    RawRec<R> y;
    if constexpr (sizeof(R) == 4) {
        y.q.x = (uint32_t)__shfl((int)x.q.x, src, 64);
        y.q.y = (uint32_t)__shfl((int)x.q.y, src, 64);
        y.q.z = (uint32_t)__shfl((int)x.q.z, src, 64);
        y.q.w = (uint32_t)__shfl((int)x.q.w, src, 64);
    } else {
        y.cell = (uint32_t)__shfl((int)x.cell, src, 64);
        y.f.x = __shfl(x.f.x, src, 64); y.f.y = __shfl(x.f.y, src, 64);
        y.v.x = __shfl(x.v.x, src, 64); y.v.y = __shfl(x.v.y, src, 64);
    }
    return y;
}

// Origin index q0 * H + (p0 mod H) of a stored record (< H * N <= 8192).
template <typename R>
__device__ __forceinline__ uint32_t raw_origin(const RawRec<R>& x, int log2H) {
    if constexpr (sizeof(R) == 4) return ((x.q.x & 0x1FFFu) << log2H) | ((x.q.x >> 13) & 0x1Fu);
    else return ((x.cell & 0xFFFFu) << log2H) | ((x.cell >> 16) & ((1u << log2H) - 1u));
}

// ---------------------------------------------------------------------------------------
// Records of each bucket grouped by tap origin.
//
// Inside one bucket (channel, plane, strip) the records are put in order of their tap origin
// o = q0 * H + (p0 mod H), o < H * N <= 8192, by a counting sort in LDS (one work-group per
// bucket).  Records with the same origin then lie next to each other, and the gridding sums
// a run of them in registers before adding it to the strip once: on 8 s integrations a
// baseline stays in one grid cell for several steps, and dense buckets hold tens of records
// per origin.
#ifndef WSIMG_SORT_UNROLL
#define WSIMG_SORT_UNROLL 8
#endif
constexpr int kOriginBins = 8192;
constexpr int kSortThreads = 512;

// One work-group per bucket (the big ones first).
template <typename R>
__global__ void __launch_bounds__(kSortThreads)
k_origin_sort(Geom g, const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ rec_cell,
              const void* __restrict__ rec, uint32_t* __restrict__ rec_cell2, void* __restrict__ rec2,
              const R* __restrict__ rec_w, R* __restrict__ rec_w2, const uint32_t* __restrict__ big,
              uint32_t big_cap, const WorkList* __restrict__ wl) {
    __shared__ uint32_t hist[kOriginBins];
    __shared__ uint32_t part[kSortThreads / 64];
    constexpr int PER = kOriginBins / kSortThreads;
    // blocks x < big_cap take the listed big buckets (dispatched first); the others take bucket
    // x - big_cap (channel * nb1 + plane * S + strip) unless it is big
    size_t b;
    if (blockIdx.x < big_cap) {
        if (blockIdx.x >= wl->n_big) return;
        b = big[blockIdx.x];
    } else {
        b = (size_t)blockIdx.x - big_cap;
    }
    const uint32_t beg = offsets[b << kLogReplicas], end = offsets[(b + 1) << kLogReplicas];
    if (blockIdx.x >= big_cap && end - beg > kBigBucket) return;
    const int t = threadIdx.x;
    if (end - beg <= 1) {
        if (end - beg == 1 && t == 0) {
            store_record<R>(rec_cell2, rec2, beg, fetch_record<R>(rec_cell, rec, beg));
            if (rec_w) rec_w2[beg] = rec_w[beg];
        }
        return;
    }
    if (end - beg <= 64) {
        // a small bucket (half the non-empty ones on an 8192^2 grid): one wave sorts it with a
        // bitonic network over the lanes, on (origin, position) so equal origins keep their
        // order; no histogram, no barrier
        if (t >= 64) return;
        const uint32_t nb = end - beg;
        RawRec<R> x{};
        R xw = (R)0;
        uint32_t key = 0xFFFFFFFFu;
        if ((uint32_t)t < nb) {
            x = fetch_record<R>(rec_cell, rec, beg + t);
            if (rec_w) xw = rec_w[beg + t];
            key = (raw_origin<R>(x, g.log2H) << 6) | (uint32_t)t;
        }
#pragma unroll
        for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                const uint32_t o = (uint32_t)__shfl_xor((int)key, stride, 64);
                const bool asc = (t & size) == 0 || size == 64, low = (t & stride) == 0;
                key = (low == asc) ? (key < o ? key : o) : (key > o ? key : o);
            }
        }
        const int src = (int)(key & 63u);
        RawRec<R> y = shfl_record<R>(x, src);
        const R yw = rec_w ? shfl_real<R>(xw, src) : (R)0;
        if ((uint32_t)t < nb) {
            store_record<R>(rec_cell2, rec2, beg + t, y);
            if (rec_w) rec_w2[beg + t] = yw;
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) hist[i * kSortThreads + t] = 0u;
    __syncthreads();
    // U records per thread in flight before their atomics (a bucket of the uv centre holds up
    // to 7e5 records, all walked by this one work-group)
    constexpr int U = WSIMG_SORT_UNROLL;
    constexpr uint32_t US = (uint32_t)U * kSortThreads;
    uint32_t r = beg + t;
    for (; r + (U - 1) * kSortThreads < end; r += US) {
        uint32_t o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) o[u] = raw_origin<R>(fetch_record<R>(rec_cell, rec, r + u * kSortThreads), g.log2H);
#pragma unroll
        for (int u = 0; u < U; ++u) atomicAdd(&hist[o[u]], 1u);
    }
    for (; r < end; r += kSortThreads)
        atomicAdd(&hist[raw_origin<R>(fetch_record<R>(rec_cell, rec, r), g.log2H)], 1u);
    __syncthreads();
    // exclusive scan of the bins: thread t owns bins [t * PER, (t + 1) * PER); the thread sums
    // are scanned within each wave by shuffles, then the wave totals are added across waves
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) { v[i] = hist[t * PER + i]; sum += v[i]; }
    const int lane = t & 63, wave = t >> 6;
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) part[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int w = 0; w < wave; ++w) run += part[w];
#pragma unroll
    for (int i = 0; i < PER; ++i) { hist[t * PER + i] = run; run += v[i]; }
    __syncthreads();
    r = beg + t;
    for (; r + (U - 1) * kSortThreads < end; r += US) {
        RawRec<R> x[U];
        R xw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x[u] = fetch_record<R>(rec_cell, rec, r + u * kSortThreads);
            xw[u] = rec_w ? rec_w[r + u * kSortThreads] : (R)0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t to = beg + atomicAdd(&hist[raw_origin<R>(x[u], g.log2H)], 1u);
            store_record<R>(rec_cell2, rec2, to, x[u]);
            if (rec_w) rec_w2[to] = xw[u];
        }
    }
    for (; r < end; r += kSortThreads) {
        const RawRec<R> x = fetch_record<R>(rec_cell, rec, r);
        const uint32_t to = beg + atomicAdd(&hist[raw_origin<R>(x, g.log2H)], 1u);
        store_record<R>(rec_cell2, rec2, to, x);
        if (rec_w) rec_w2[to] = rec_w[r];
    }
}

// ---------------------------------------------------------------------------------------
// Work-group shapes, fixed per (precision, image size).  Each FFT runs on a base radix
// 2^LR (2^LR elements per thread between LDS exchanges); the base radix of each pass and
// the stacking block sizes are build-time choices (WSIMG_<precision>_LR1/_LR2/_PX2/_BS), picked
// by measurement.
//   pass 1: H grid rows per strip; the strip accumulates in float64 (16 B per cell) whatever
//           the precision, so H * N <= 8192 cells; NT1 = H * N / 2^LR1 threads;
//   pass 2: the intermediate's column blocks hold B columns, B * N = PX2 pixels; a stacking
//           block takes BS <= B of them with NT2 = BS * N / 2^LR2 threads.
#ifndef WSIMG_F32_LR1
#define WSIMG_F32_LR1 4
#endif

// float stacking, per image size (log2 n): radix 16 at 4096^2 (1.16 ms against 1.26 ms with
// radix 8 for 32 planes), radix 8 at 8192^2 (64 planes: 12.3 ms against 14.3 ms; 1024 threads of
// 8 pixels keep 4 waves per SIMD where 512 threads of 16 pixels kept 2) and below 4096^2
// (1024^2: 1.92 ms against 2.18 ms for 64 channels of 16 planes).  WSIMG_F32_LR2_N<log2 n>
// sets one size (the autotuner's per-shape choices); WSIMG_F32_LR2 overrides every size.
#ifndef WSIMG_F32_LR2_N12
#define WSIMG_F32_LR2_N12 4
#endif
#ifndef WSIMG_F32_LR2_N13
#define WSIMG_F32_LR2_N13 3
#endif
#ifndef WSIMG_F32_LR2_SMALL
#define WSIMG_F32_LR2_SMALL 3
#endif
template <int LOG2N> constexpr int f32_stack_radix_log2() {
#ifdef WSIMG_F32_LR2
    return WSIMG_F32_LR2;
#else
#ifdef WSIMG_F32_LR2_N4
    if (LOG2N == 4) return WSIMG_F32_LR2_N4;
#endif
#ifdef WSIMG_F32_LR2_N5
    if (LOG2N == 5) return WSIMG_F32_LR2_N5;
#endif
#ifdef WSIMG_F32_LR2_N6
    if (LOG2N == 6) return WSIMG_F32_LR2_N6;
#endif
#ifdef WSIMG_F32_LR2_N7
    if (LOG2N == 7) return WSIMG_F32_LR2_N7;
#endif
#ifdef WSIMG_F32_LR2_N8
    if (LOG2N == 8) return WSIMG_F32_LR2_N8;
#endif
#ifdef WSIMG_F32_LR2_N9
    if (LOG2N == 9) return WSIMG_F32_LR2_N9;
#endif
#ifdef WSIMG_F32_LR2_N10
    if (LOG2N == 10) return WSIMG_F32_LR2_N10;
#endif
#ifdef WSIMG_F32_LR2_N11
    if (LOG2N == 11) return WSIMG_F32_LR2_N11;
#endif
    return LOG2N == 13 ? WSIMG_F32_LR2_N13 : (LOG2N == 12 ? WSIMG_F32_LR2_N12 : WSIMG_F32_LR2_SMALL);
#endif
}
// base radix of the prediction's column pass (the stacking pass's transpose)
#ifndef WSIMG_F32_LR2A
#define WSIMG_F32_LR2A 3
#endif
#ifndef WSIMG_F64_LR2A
#define WSIMG_F64_LR2A 3
#endif
#ifndef WSIMG_F64_LR1
#define WSIMG_F64_LR1 4
#endif
#ifndef WSIMG_F64_LR2
#define WSIMG_F64_LR2 3
#endif
// cells of one gridding strip (H * N): its float64 accumulator takes 16 B per cell of LDS.
// Images below 4096^2 use the smaller strip (two work-groups per CU, fewer walks per strip).
#ifndef WSIMG_STRIP_CELLS
#define WSIMG_STRIP_CELLS 8192
#endif
#ifndef WSIMG_STRIP_CELLS_SMALL
#define WSIMG_STRIP_CELLS_SMALL 4096
#endif
// grid rows per strip below 4096^2 when > 0 (instead of STRIP_CELLS_SMALL / N, at most 4).
// Two, the walk's register rows for W <= 7, so that a record visit decodes its record once:
// 64 channels of 1024^2 10.0 -> 9.45 ms, 256^2 0.51 -> 0.36 ms, 2048^2 unchanged
#ifndef WSIMG_STRIP_ROWS_SMALL
#define WSIMG_STRIP_ROWS_SMALL 2
#endif
// WSIMG_STRIP_ROWS_N<log2 n> (n < 4096) sets one size (the autotuner's per-shape choices; 0:
// by cells, at most 4).  64 channels of 1024^2 grid in 3.8 ms with two rows against 4.4 ms with
// four.
template <int LOG2N> constexpr int strip_rows_small() {
#ifdef WSIMG_STRIP_ROWS_N8
    if (LOG2N == 8) return WSIMG_STRIP_ROWS_N8;
#endif
#ifdef WSIMG_STRIP_ROWS_N9
    if (LOG2N == 9) return WSIMG_STRIP_ROWS_N9;
#endif
#ifdef WSIMG_STRIP_ROWS_N10
    if (LOG2N == 10) return WSIMG_STRIP_ROWS_N10;
#endif
#ifdef WSIMG_STRIP_ROWS_N11
    if (LOG2N == 11) return WSIMG_STRIP_ROWS_N11;
#endif
    return WSIMG_STRIP_ROWS_SMALL;
}
static_assert(WSIMG_STRIP_CELLS <= 8192 && WSIMG_STRIP_CELLS_SMALL <= 8192,
              "origins of a strip index an 8192-bin histogram");
#ifndef WSIMG_F32_PX2
#define WSIMG_F32_PX2 8192
#endif
#ifndef WSIMG_F64_PX2
#define WSIMG_F64_PX2 4096
#endif
// Per image size: at 8192^2 a strip is one grid row, and with one column per layout block each
// row element went to its own 64 KB-strided address (8-byte stores: 32 GB written for 9.3 GB of
// strips on the LOFAR-shaped image).  Eight float columns per block make every row store a
// whole 64-byte segment (gridding 28.9 -> 20.8 ms, stacking 12.1 -> 13.9 ms as each stacking
// block now reads 8 of every 64 bytes: 47.7 -> 41.4 ms per image; 2, 4 and 16 columns: 45.9,
// 43.3, 43.4 ms).  In double, 1, 2, 4 and 8 columns time alike (101-104 ms): one is kept.
#ifndef WSIMG_F32_PX2_N13
#define WSIMG_F32_PX2_N13 65536
#endif
#ifndef WSIMG_F64_PX2_N13
#define WSIMG_F64_PX2_N13 8192
#endif
#ifndef WSIMG_F32_PX2_N12
#define WSIMG_F32_PX2_N12 WSIMG_F32_PX2
#endif
#ifndef WSIMG_F64_PX2_N12
#define WSIMG_F64_PX2_N12 WSIMG_F64_PX2
#endif
template <typename R, int LOG2N> constexpr int layout_pixels() {
    if constexpr (sizeof(R) == 4) return LOG2N == 13 ? WSIMG_F32_PX2_N13 : (LOG2N == 12 ? WSIMG_F32_PX2_N12 : WSIMG_F32_PX2);
    else return LOG2N == 13 ? WSIMG_F64_PX2_N13 : (LOG2N == 12 ? WSIMG_F64_PX2_N12 : WSIMG_F64_PX2);
}
// image columns per stacking block (0: all B columns of a layout block).  float: one, so that
// several blocks share a CU and one block's barriers overlap another's work (a 4096^2 image
// of 32 planes: 1.44 -> 1.26 ms with radix-8 passes, 1.18 ms with radix 16: 256 threads per
// block, two blocks per CU)
#ifndef WSIMG_F32_BS
#define WSIMG_F32_BS 1
#endif
#ifndef WSIMG_F64_BS
#define WSIMG_F64_BS 0
#endif
// 1: stacking blocks that share layout blocks are placed on one XCD (below)
#ifndef WSIMG_COLS_XCD_MAP
#define WSIMG_COLS_XCD_MAP 1
#endif


// bytes of the stacking pass's LDS plane-flag table: the largest plane count a plan takes
constexpr size_t kPlaneTab = 4096;

template <typename R, int LOG2N> struct Shape {
    static constexpr int N = 1 << LOG2N;
    // base radices (log2), at most log2(N) - 1 so that a transform has two passes or more
    static constexpr int LR1_0 = sizeof(R) == 4 ? WSIMG_F32_LR1 : WSIMG_F64_LR1;
    static constexpr int LR2_0 = sizeof(R) == 4 ? f32_stack_radix_log2<LOG2N>() : WSIMG_F64_LR2;
    static constexpr int LR1 = LR1_0 < LOG2N ? LR1_0 : LOG2N - 1;
    static constexpr int LR2 = LR2_0 < LOG2N ? LR2_0 : LOG2N - 1;
    static constexpr int E1 = 1 << LR1, E2 = 1 << LR2;
    static constexpr int LR2A_0 = sizeof(R) == 4 ? WSIMG_F32_LR2A : WSIMG_F64_LR2A;
    static constexpr int LR2A = LR2A_0 < LOG2N ? LR2A_0 : LOG2N - 1;
    static constexpr int CAP1 = LOG2N >= 12 ? WSIMG_STRIP_CELLS : WSIMG_STRIP_CELLS_SMALL;
    // a row at least; at most 4, so that small images still have many strips in flight and
    // few register walks per strip (a 256^2 image: 1.18 ms with 16-row strips)
    static constexpr int HS = strip_rows_small<LOG2N>();
    static constexpr int H0 = (LOG2N < 12 && HS > 0) ? HS
                              : (CAP1 / N < 4 ? (CAP1 / N < 1 ? 1 : CAP1 / N) : 4);
    static constexpr int H = H0 < N / 2 ? H0 : N / 2;
    static constexpr int NT1 = (H * N / E1) < 64 ? 64 : (H * N / E1);
    static constexpr int PX2 = layout_pixels<R, LOG2N>();
    // the intermediate holds B columns side by side per row (the gridding pass's write unit); a
    // stacking block takes BS <= B of them and a prediction column block BA <= B
    static constexpr int B0 = PX2 / N < N / 2 ? PX2 / N : N / 2;   // at most half a (padded) grid
    static constexpr int B = B0 < 1 ? 1 : B0;
    // the column blocks the work-groups of the column passes can hold in LDS
    static constexpr int PXA = sizeof(R) == 4 ? WSIMG_F32_PX2 : WSIMG_F64_PX2;
    static constexpr int BA0 = PXA / N < 1 ? 1 : PXA / N;
    static constexpr int BA = BA0 < B ? BA0 : B;
    static constexpr int BS0 = sizeof(R) == 4 ? WSIMG_F32_BS : WSIMG_F64_BS;
    static constexpr int BS = BS0 <= 0 ? BA : (BS0 > B ? B : BS0);
    static_assert((BS & (BS - 1)) == 0 && (BA & (BA - 1)) == 0, "column blocks: powers of two");
    static constexpr int NT2 = (BS * N / E2) < 64 ? 64 : (BS * N / E2);   // stacking
    static constexpr int NT2A = (BA * N >> LR2A) < 64 ? 64 : (BA * N >> LR2A);   // prediction column pass
    static constexpr int LDS1 = lds_padded_elems_c(H * N);                 // elements
    static constexpr size_t LDS1_BYTES = (size_t)LDS1 * sizeof(double2);   // float64 accumulation
    static constexpr int LDS2 = lds_padded_elems_c(BA * N);                // complex elements
    static constexpr size_t LDS2_BYTES = (size_t)LDS2 * 2 * sizeof(R);      // column pass of prediction
    static constexpr int LDS2S = lds_padded_elems_c(BS * N);               // stacking FFT buffer
    static constexpr size_t LDS2S_BUF = (size_t)LDS2S * 2 * sizeof(R);
    // the per-pixel n - 1 table goes to LDS when it fits beside the FFT buffer and the plane
    // flags (kPlaneTab bytes, after everything else), else it stays in registers
    static constexpr bool NM1_LDS = LDS2S_BUF + sizeof(double) * E2 * NT2 + kPlaneTab <= 160 * 1024;
    static constexpr size_t PTAB_OFF = LDS2S_BUF + (NM1_LDS ? sizeof(double) * E2 * NT2 : 0);
    static constexpr size_t LDS2S_BYTES = PTAB_OFF + kPlaneTab;
};

// ---------------------------------------------------------------------------------------
// gridding (+ row FFT) of one (plane, strip) in LDS

// The strip's cells accumulate in float64 in LDS for both precisions: with no grid padding
// the taper division amplifies grid rounding near the image edge by up to 1/C(1/2)^2 (about
// 2500 for W = 7), and float32 atomic accumulation alone costs ~1e-5 of the image there.
// The per-tap products are formed in the plan's precision; the float path converts the
// strip to float32 in place before its FFT.
//
// Each lane walks a chunk of consecutive records (records are in (bucket, origin) order) for
// RW grid rows of the strip at a time, summing the taps of a run of equal-origin records in
// float64 registers (RW x WMAX complex values; each tap product is still formed in the plan
// precision, so the sums match per-tap float64 accumulation up to order) and adding them to
// the LDS strip when the origin changes or the chunk ends.  (Float32 run sums cost up to
// 4e-6 of the image peak near the edges, where the taper amplifies grid rounding.)  The chunk length grows with the records the
// strip reads (one record per lane up to NT records, at most chunk_max<R>()), so sparse strips
// keep every lane busy and dense ones merge long runs.  Float records take chunks of up to 64
// (8192^2 LOFAR-shaped gridding 16.2 -> 15.6 ms against 16; 4096^2 0.95 -> 0.93 ms), float64
// ones of up to 16 (64 made the same 8192^2 float64 gridding 40.5 -> 41.4 ms).
#ifndef WSIMG_GRID_BATCH
#define WSIMG_GRID_BATCH 4
#endif
#ifndef WSIMG_F32_GRID_CHUNK_MAX
#define WSIMG_F32_GRID_CHUNK_MAX 64
#endif
#ifndef WSIMG_F64_GRID_CHUNK_MAX
#define WSIMG_F64_GRID_CHUNK_MAX 16
#endif
template <typename R> constexpr uint32_t chunk_max() {
    return sizeof(R) == 4 ? WSIMG_F32_GRID_CHUNK_MAX : WSIMG_F64_GRID_CHUNK_MAX;
}

// Register rows per walk for a support class WMAX: the float64 run sums (4 VGPRs per tap)
// stay within WSIMG_WALK_VGPRS registers.
#ifndef WSIMG_WALK_VGPRS
#define WSIMG_WALK_VGPRS 64
#endif
template <typename R, int WMAX> struct WalkRows {
    static constexpr int words = WMAX * 4;
    static constexpr int fit = WSIMG_WALK_VGPRS / words;
    static constexpr int value = fit >= 8 ? 8 : (fit >= 4 ? 4 : (fit >= 2 ? 2 : 1));
};

// One occupied strip (plane k of channel c, strip s) by the whole work-group.
// aux: the list entry's companion word (parts = 1 when not split); split_acc / split_done:
// the slots of split strips (float64 strip sums, completed-part counters).
template <typename R, bool FFT, int LOG2N, int WMAX>
__device__ __forceinline__ void grid_strip(const Geom& g, int c, int k, int s, unsigned char* smem_raw,
                                           const uint32_t* __restrict__ offsets,
                                           const uint32_t* __restrict__ rec_cell,
                                           const void* __restrict__ rec,
                                           const R* __restrict__ kbc, const typename Cx<R>::T* __restrict__ tw,
                                           typename Cx<R>::T* __restrict__ out, const R* __restrict__ kbw,
                                           const R* __restrict__ recw, uint32_t aux = 1u,
                                           double2* __restrict__ split_acc = nullptr,
                                           uint32_t* __restrict__ split_done = nullptr) {
    using C = typename Cx<R>::T;
    using SH = Shape<R, LOG2N>;
    constexpr int n = SH::N, H = SH::H, NT = SH::NT1, nmask = n - 1;
    constexpr int LOG2H = Log2Of<H>::value_any;
    constexpr int elems = H * n;
    constexpr int RW = WalkRows<R, WMAX>::value < H ? WalkRows<R, WMAX>::value : H;
    constexpr int NG = H / RW, LOG2NG = Log2Of<NG>::value_any;
    double2* acc = reinterpret_cast<double2*>(smem_raw);
    C* lds = reinterpret_cast<C*>(smem_raw);
    const int tid = threadIdx.x;
    const int row0 = s * H;
    for (int e = tid; e < SH::LDS1; e += NT) acc[e] = make_double2(0.0, 0.0);
    __syncthreads();

    const int W = g.support, hW = g.half;
    constexpr int TC = WMAX / 2;               // centre slot of the tap arrays
    int s_lo = (row0 - (W - 1)) >> LOG2H;
    if (s_lo < 0) s_lo = 0;
    constexpr int shift = FFT ? (n >> 1) : 0;   // place cell q at (q + n/2) mod n: the centring
    const uint32_t parts = aux & 0xFFu, part = (aux >> 8) & 0xFFu, slot = aux >> 16;
    // the rows of plane kk reach plane k: kk = k, or kk = k - Ww + 1 .. k with the w-kernel,
    // whose rows then carry the weight of their w-tap wj = k - kk (split strips: one plane)
    const int klo = g.wsup ? (k - g.wsup + 1 < 0 ? 0 : k - g.wsup + 1) : k;
    for (int kk = klo; kk <= k; ++kk) {
        const int wj = k - kk;
        const int bucket0 = c * g.nb1 + kk * g.S;
        uint32_t vbeg = offsets[(size_t)(bucket0 + s_lo) << kLogReplicas];
        uint32_t vend = offsets[(size_t)(bucket0 + s + 1) << kLogReplicas];
        if (parts > 1) {       // this part's share of the strip's records
            const uint64_t len = vend - vbeg;
            const uint32_t pb = vbeg + (uint32_t)(len * part / parts), pe = vbeg + (uint32_t)(len * (part + 1) / parts);
            vbeg = pb;
            vend = pe;
        }
        const uint32_t nv = vend - vbeg;
        // records per walk item: the fewest for which the strip's items (chunks x row groups)
        // fit in one pass of the work-group (rounding down left e.g. 4260 records of a 512-thread
        // group in 533 chunks of 8: two rounds, the second for 21 threads)
        uint32_t chunk = (uint32_t)(((uint64_t)nv * NG + NT - 1) / NT);
        chunk = chunk < 1u ? 1u : (chunk > chunk_max<R>() ? chunk_max<R>() : chunk);
        const uint32_t items = ((nv + chunk - 1) / chunk) << LOG2NG;

        for (uint32_t it = tid; it < items; it += NT) {
            const int rlo = row0 + (int)(it & (NG - 1)) * RW;     // first grid row of this walk
            uint32_t r = vbeg + (it >> LOG2NG) * chunk;
            const uint32_t re = r + chunk < vend ? r + chunk : vend;
            int sp = s_lo;
            uint32_t bend = offsets[(size_t)(bucket0 + sp + 1) << kLogReplicas];
            // run sums and tap weights by centred tap slot t = C + d (tap a = h + d, |d| <= h)
            double2 sum[RW][WMAX];
#pragma unroll
            for (int rr = 0; rr < RW; ++rr)
#pragma unroll
                for (int t = 0; t < WMAX; ++t) sum[rr][t] = make_double2(0.0, 0.0);
            int cq = -1, cp = 0;
            // dirty: the sums hold a run not yet added to the strip.  A flush leaves the sums as
            // they are; the next record that adds taps scales them by 0 (keep) in the same fused
            // multiply-add, so no lane zeroes registers on its own.
            bool dirty = false;
            auto flush = [&]() {
                if (!dirty) return;
                dirty = false;
#pragma unroll
                for (int rr = 0; rr < RW; ++rr) {
                    const int b = rlo + rr - cp;
                    if ((unsigned)b < (unsigned)W) {
                        const int lrow = (rlo + rr - row0) << LOG2N;
                        const int q_c = cq + hW + shift - TC;      // cell of slot t: q_c + t
#pragma unroll
                        for (int t = 0; t < WMAX; ++t) {
                            if (t - TC <= hW && TC - t <= hW) {
                                double2* dst = &acc[lds_pad(lrow + ((q_c + t) & nmask))];
                                atomicAdd(&dst->x, sum[rr][t].x);
                                atomicAdd(&dst->y, sum[rr][t].y);
                            }
                        }
                    }
                }
            };
            // one record: bucket tracking, run bookkeeping and its taps in this walk
            auto process = [&](const RawRec<R>& x, uint32_t r) {
                while (r >= bend) {
                    ++sp;
                    bend = offsets[(size_t)(bucket0 + sp + 1) << kLogReplicas];
                }
                int q0, p0;
                C fr, v;
                decode_record<R>(x, sp, LOG2H, q0, p0, fr, v);
                if (recw) {     // the w-kernel's weight of this row on plane k
                    const R gw = kb_tap<R>(kbw, wj, recw[r]);
                    v.x *= gw;
                    v.y *= gw;
                }
                if (q0 != cq || p0 != cp) {
                    flush();
                    cq = q0;
                    cp = p0;
                }
                if (rlo + RW - 1 < p0 || rlo > p0 + W - 1) return;       // no tap row in this walk
                R gx[WMAX];
                kb_taps_centred<R, WMAX>(kbc, hW, fr.x, gx);
                // every row of the walk, with zero weight on the rows the record does not reach
                const double keep = dirty ? 1.0 : 0.0;
                dirty = true;
#pragma unroll
                for (int rr = 0; rr < RW; ++rr) {
                    const int b = rlo + rr - p0;
                    const bool reach = (unsigned)b < (unsigned)W;
                    const R gy = reach ? kb_tap<R>(kbc, reach ? b : 0, fr.y) : (R)0;
                    const R vr = v.x * gy, vi = v.y * gy;
#pragma unroll
                    for (int t = 0; t < WMAX; ++t) {
                        if (t - TC <= hW && TC - t <= hW) {
                            sum[rr][t].x = __builtin_fma(sum[rr][t].x, keep, (double)(vr * gx[t]));
                            sum[rr][t].y = __builtin_fma(sum[rr][t].y, keep, (double)(vi * gx[t]));
                        }
                    }
                }
            };
            // records are fetched WSIMG_GRID_BATCH at a time, so that several loads are in flight
            constexpr uint32_t KB = WSIMG_GRID_BATCH;
            for (uint32_t left = re - r; left > 0;) {
                const uint32_t cnt = left < KB ? left : KB;
                RawRec<R> buf[KB];
#pragma unroll
                for (uint32_t i = 0; i < KB; ++i)
                    if (i < cnt) buf[i] = fetch_record<R>(rec_cell, rec, r + i);
#pragma unroll
                for (uint32_t i = 0; i < KB; ++i)
                    if (i < cnt) process(buf[i], r + i);
                r += cnt;
                left -= cnt;
            }
            flush();
        }
    }
    __syncthreads();

    if (parts > 1) {
        // add this part into the strip's slot; the work-group completing the last part takes
        // the sum (and leaves the slot and its counter zero for the next call)
        __shared__ int s_last;
        double2* gacc = split_acc + (size_t)slot * SH::LDS1;
        for (int e = tid; e < SH::LDS1; e += NT) {
            const double2 a = acc[e];
            if (a.x != 0.0) unsafeAtomicAdd(&gacc[e].x, a.x);
            if (a.y != 0.0) unsafeAtomicAdd(&gacc[e].y, a.y);
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) s_last = atomicAdd(&split_done[slot], 1u) == parts - 1 ? 1 : 0;
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        unsigned long long* gbits = reinterpret_cast<unsigned long long*>(gacc);
        for (int e = tid; e < SH::LDS1; e += NT) {
            acc[e] = make_double2(__longlong_as_double((long long)atomicExch(&gbits[2 * e], 0ull)),
                                  __longlong_as_double((long long)atomicExch(&gbits[2 * e + 1], 0ull)));
        }
        if (tid == 0) atomicExch(&split_done[slot], 0u);
        __syncthreads();
    }

    if constexpr (FFT) {
        if constexpr (sizeof(R) == 4) {
            // float64 strip -> float32 strip in the same LDS, in two halves: the floats of the
            // first half land on doubles this half reads (so a barrier between read and write),
            // those of the second half on doubles the first half already consumed.
            constexpr int HALF = elems / 2;
            constexpr int PER = (HALF + NT - 1) / NT;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double2 t[PER];
#pragma unroll
                for (int i = 0; i < PER; ++i) {
                    const int e = h * HALF + tid + i * NT;
                    if (tid + i * NT < HALF) t[i] = acc[lds_pad(e)];
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < PER; ++i) {
                    const int e = h * HALF + tid + i * NT;
                    if (tid + i * NT < HALF) lds[lds_pad(e)] = cmake<C>((R)t[i].x, (R)t[i].y);
                }
                __syncthreads();
            }
        }
        fft_rows_lds<LOG2N, SH::LR1, H, NT>(lds, tw);
        // column-block layout [k][jb][p'][B], p' = (p + n/2) mod n: the next pass reads a
        // contiguous [n][B] block per plane.  Image column j takes FFT bin (j + n/2) mod n.
        // only the image's columns are kept (the crop of a padded grid)
        constexpr int B = SH::B, LOG2B = Log2Of<B>::value_any;
        const int pp0 = (row0 + (n >> 1)) & nmask;
        C* dst = out + (size_t)(c * g.nw + k) * g.plane_elems;
        constexpr int LHB = LOG2H + LOG2B;
        const int out_elems = H * g.n_img;
        for (int e = tid; e < out_elems; e += NT) {
            const int jb = e >> LHB;
            const int rem = e & ((1 << LHB) - 1);
            const int lr = rem >> LOG2B, col = rem & (B - 1);
            const int jp = (g.crop + (jb << LOG2B) + col + (n >> 1)) & nmask;
            dst[(((size_t)jb << LOG2N) + pp0 + lr) * B + col] = lds[lds_pad((lr << LOG2N) + jp)];
        }
    } else {
        C* dst = out + ((size_t)(c * g.nw + k) << (2 * LOG2N)) + ((size_t)row0 << LOG2N);
        for (int e = tid; e < elems; e += NT) {
            const double2 a = acc[lds_pad(e)];
            dst[e] = cmake<C>((R)a.x, (R)a.y);
        }
    }
}

// Next entry of the strip work list for a persistent work-group (one thread asks; -1: none
// left).  Heavy entries (and split parts) go to whichever work-group asks first.  The light
// entries lie in bucket order within the chunks of consecutive strips k_occupancy writes; they
// are cut into 8 contiguous ranges, one per XCD (work-groups go to the XCDs round-robin, so
// work-group x runs on XCD x mod 8), and the work-groups of an XCD take its range in order: the
// strips an XCD grids at the same time are neighbours, whose records (a record's taps reach
// (W + H - 2) / H + 1 strips) its L2 then serves to all of them.  An XCD whose range is done
// takes entries from the others' ranges.  The asking thread keeps a mask of the sources it has
// found exhausted (bit 8: the heavy entries), so that a work-group that has moved on to other
// ranges does not ask the spent counters again (each question is an agent-scope load past the
// XCD's L2: 4% of the gridding of 64 channels of 1024^2, whose strips take tens of us each),
// and the list's two lengths are read once per work-group.
// (One global counter over the whole list, the earlier scheme, gridded the 8192^2 LOFAR-shaped
// image in 19.3 ms against 17.7 ms, and 4096^2 in 1.13 against 1.09 ms.)
__device__ __forceinline__ int fetch_item(WorkList* __restrict__ wl, const uint32_t* __restrict__ list,
                                          const uint32_t* __restrict__ list_aux, uint32_t list_cap,
                                          unsigned n_heavy, unsigned n_light, uint32_t& aux, uint32_t& spent) {
    aux = 1u;
    if (!(spent & 0x100u)) {
        if (__hip_atomic_load(&wl->next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n_heavy) {
            const unsigned i = atomicAdd(&wl->next, 1u);
            if (i < n_heavy) { aux = list_aux[i]; return (int)list[i]; }
        }
        spent |= 0x100u;
    }
    const int x0 = (int)(blockIdx.x & 7u);
    for (int t = 0; t < 8; ++t) {
        const int x = (x0 + t) & 7;
        if (spent & (1u << x)) continue;
        const unsigned lo = (unsigned)(((uint64_t)n_light * (unsigned)x) >> 3);
        const unsigned hi = (unsigned)(((uint64_t)n_light * (unsigned)(x + 1)) >> 3);
        if (__hip_atomic_load(&wl->xnext[x].n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < hi - lo) {
            const unsigned j = atomicAdd(&wl->xnext[x].n, 1u);
            if (j < hi - lo) return (int)list[list_cap - 1 - (lo + j)];
        }
        spent |= 1u << x;
    }
    return -1;
}

// The gridding step alone: work-group (b, c) = strip b of every plane of channel c; empty
// strips are zeroed.
template <typename R, int LOG2N, int WMAX>
__global__ void __launch_bounds__((Shape<R, LOG2N>::NT1))
k_grid_only(Geom g, const uint32_t* __restrict__ offsets, const uint8_t* __restrict__ occ,
            const uint32_t* __restrict__ rec_cell, const void* __restrict__ rec, const R* __restrict__ kbc,
            typename Cx<R>::T* __restrict__ out, const R* __restrict__ kbw, const R* __restrict__ recw) {
    using C = typename Cx<R>::T;
    using SH = Shape<R, LOG2N>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int c = blockIdx.y, b = blockIdx.x;
    const int k = b / g.S, s = b - k * g.S;
    if (!occ[c * g.nb1 + b]) {
        C* dst = out + ((size_t)(c * g.nw + k) << (2 * LOG2N)) + ((size_t)(s * SH::H) << LOG2N);
        for (int e = threadIdx.x; e < SH::H * SH::N; e += SH::NT1) dst[e] = cmake<C>((R)0, (R)0);
        return;
    }
    grid_strip<R, false, LOG2N, WMAX>(g, c, k, s, smem_raw, offsets, rec_cell, rec, kbc, nullptr, out, kbw, recw);
}

// Gridding + row FFT: a persistent grid walks the work list of occupied strips of all
// channels (heavy ones first) through an atomic counter; every work-group leaves once the
// list is exhausted.
template <typename R, int LOG2N, int WMAX>
__global__ void __launch_bounds__((Shape<R, LOG2N>::NT1))
k_grid_rows(Geom g, WorkList* __restrict__ wl, const uint32_t* __restrict__ list,
            const uint32_t* __restrict__ list_aux, uint32_t list_cap,
            const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ rec_cell,
            const void* __restrict__ rec, const R* __restrict__ kbc, const typename Cx<R>::T* __restrict__ tw,
            typename Cx<R>::T* __restrict__ out, double2* __restrict__ split_acc,
            uint32_t* __restrict__ split_done, const R* __restrict__ kbw, const R* __restrict__ recw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int item;
    __shared__ uint32_t item_aux;
    uint32_t spent = 0u;        // thread 0's mask of exhausted work-list sources
    unsigned n_heavy = 0u, n_light = 0u;
    if (threadIdx.x == 0) { n_heavy = wl->n_heavy; n_light = wl->n_light; }
    while (true) {
        if (threadIdx.x == 0) {
            uint32_t x = 1u;
            item = fetch_item(wl, list, list_aux, list_cap, n_heavy, n_light, x, spent);
            item_aux = x;
        }
        __syncthreads();
        const int b = item;
        const uint32_t aux = item_aux;
        __syncthreads();
        if (b < 0) break;
        const int c = b / g.nb1, bb = b - c * g.nb1;
        const int k = bb / g.S, s = bb - k * g.S;
        grid_strip<R, true, LOG2N, WMAX>(g, c, k, s, smem_raw, offsets, rec_cell, rec, kbc, opaque_ptr(tw), out,
                                         kbw, recw, aux, split_acc, split_done);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// column FFTs, w-phase, stacking over planes, taper
//
// Work-group = one block of BS image columns (of a layout block of B), E = 2^LR2 pixels per
// thread.  Per occupied plane:
//   * the inputs of the first radix-E pass come straight from HBM into registers (thread
//     tid = b * BS + c takes column c at rows b + m N/E of the plane's [n][B] layout block);
//     rows of empty strips read as 0, by the thread's packed strip flags (k_stack_flags),
//     which are loaded two occupied planes ahead;
//   * the middle passes run in LDS, the last pass leaves its outputs in registers;
//   * each output is multiplied by exp(+2 pi i w_k (n - 1)) and its real part summed over
//     planes (Kahan-compensated in float, plain in double);
//   * in float, the next plane's first-pass inputs are loaded while this plane is transformed.
// At the end: divide by the taper on both axes and by the sum of weights.

// float: the next plane's first-pass inputs are loaded while this plane is transformed
#ifndef WSIMG_COLS_PREFETCH
#define WSIMG_COLS_PREFETCH 1
#endif
template <typename R> struct Pass2Prefetch { static constexpr bool value = sizeof(R) == 4 && WSIMG_COLS_PREFETCH; };

// The stacking pass's strip flags: for channel c, plane k and b < N / 2^LR, bit m of
// flags[(c nw + k) N/2^LR + b] is set when row b + m N/2^LR of the plane lies in an occupied
// strip.  A stacking thread's first pass reads rows b + m N/2^LR (m < 2^LR), so one load per
// plane gives it the flags of all of them.
__global__ void __launch_bounds__(256)
k_stack_flags(Geom g, int nch, int lr, const uint8_t* __restrict__ occ, uint16_t* __restrict__ flags) {
    const int nr = g.n >> lr;
    const int64_t total = (int64_t)nch * g.nw * nr;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = (int)(i % nr);
    const uint8_t* o = occ + (i / nr) * g.S;
    uint32_t bits = 0;
    for (int m = 0; m < (1 << lr); ++m) bits |= (o[(b + m * nr) >> g.log2H] ? 1u : 0u) << m;
    flags[i] = (uint16_t)bits;
}

// The rows of occupied strips (zero elsewhere) of one plane's block: src is the block's
// first element in the intermediate, toff the thread's element of row b (b B + its column), fl
// the thread's flag word of the plane.  Slot m holds
// row (b + m N/2^LR + N/2) mod N, i.e. flag bit (m + 2^LR / 2) mod 2^LR.
template <typename R, int LOG2N, int LR, int B>
__device__ __forceinline__ void pass2_data(const typename Cx<R>::T* __restrict__ src, uint32_t fl,
                                           uint32_t toff, typename Cx<R>::T* x) {
    using C = typename Cx<R>::T;
    constexpr int E = 1 << LR, nr = (1 << LOG2N) >> LR;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        x[m] = cmake<C>((R)0, (R)0);
        if (fl & (1u << ((m + E / 2) & (E - 1)))) x[m] = src[(uint32_t)(m * nr * B) + toff];
    }
}

// Waves per SIMD the stacking kernel is compiled for (0: the compiler's choice; 4 caps its
// registers at 128, for two 512-thread blocks per CU with a radix-8 pass).
#ifndef WSIMG_F32_COLS_WAVES_PER_EU
#define WSIMG_F32_COLS_WAVES_PER_EU 0
#endif
#ifndef WSIMG_F64_COLS_WAVES_PER_EU
#define WSIMG_F64_COLS_WAVES_PER_EU 0
#endif
template <typename R> struct ColsWaves {
    static constexpr int value = sizeof(R) == 4 ? WSIMG_F32_COLS_WAVES_PER_EU : WSIMG_F64_COLS_WAVES_PER_EU;
};

// Stacking block index -> block of BS image columns.  Work-groups go to the 8 XCDs round-robin
// (block bid to XCD bid mod 8, as its slot bid / 8 there), so a group of Q consecutive column
// blocks is given Q consecutive slots of one XCD: they run at the same time on that XCD, and
//   * the G = B / BS blocks that read the same layout blocks of the intermediate (each B-column
//     row chunk) find the chunks the first of them fetched in the XCD's L2;
//   * the image rows they write (BS columns each, at the end) merge into whole cache lines in
//     the L2 before they reach HBM: Q blocks cover 128 bytes of every image row.
// Q is a multiple of G, so a layout block's readers stay in one group.
template <typename R, int G, int BS> __device__ __forceinline__ int stack_block(int bid, int nblk) {
    constexpr int Q0 = 128 / (int)sizeof(R) / BS;
    constexpr int Q = WSIMG_COLS_XCD_MAP ? (Q0 > G ? Q0 : G) : 1;
    if constexpr (Q <= 1) {
        return bid;
    } else {
        if (nblk % (8 * Q) != 0) return bid;
        const int xcd = bid & 7, slot = bid >> 3;
        return ((((slot / Q) << 3) + xcd) * Q) + (slot % Q);
    }
}

// PAD: the grid is padded (the image is its central crop); without it the crop logic folds away.
// CPLX: the image is complex, S / (sum W C(xi_i) C(xi_j)), interleaved (re, im) per pixel;
// the imaginary part is stacked like the real part (Kahan-compensated in float).
template <typename R, int LOG2N, bool PAD, bool CPLX>
__global__ void __launch_bounds__((Shape<R, LOG2N>::NT2), (ColsWaves<R>::value))
k_cols_stack(Geom g, const Scalars* __restrict__ sc, const uint16_t* __restrict__ sflags,
             const uint8_t* __restrict__ plane_occ, const typename Cx<R>::T* __restrict__ inter,
             const typename Cx<R>::T* __restrict__ tw, const R* __restrict__ inv_taper,
             R* __restrict__ image) {
    using C = typename Cx<R>::T;
    using SH = Shape<R, LOG2N>;
    constexpr int n = SH::N, nmask = n - 1, hn = n >> 1;
    // B: columns per layout block of the intermediate; BS: columns of this block
    constexpr int B = SH::B, BS = SH::BS, NT = SH::NT2, LOG2B = Log2Of<B>::value_any;
    constexpr int LOG2BS = Log2Of<BS>::value_any;
    constexpr int elems = BS * n;
    constexpr int LR = SH::LR2, E = SH::E2;
    static_assert(LOG2N > LR, "image side must exceed the base radix");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* lds0 = reinterpret_cast<C*>(smem_raw);
    // n - 1 of each output slot: in LDS after the FFT buffer (nm1s[s * NT + tid]) when it
    // fits there, else in registers
    double* nm1s = reinterpret_cast<double*>(lds0 + SH::LDS2S);
    double nm1r[SH::NM1_LDS ? 1 : E];
    nm1r[0] = 0.0;
    const int jb = stack_block<R, B / BS, BS>(blockIdx.x, gridDim.x), c = blockIdx.y;
    const int crop = PAD ? g.crop : 0, nimg = PAD ? g.n_img : n;
    const int tid = threadIdx.x;
    // every thread takes part in the first pass unless the block was widened to a wave
    const bool first_active = (NT == (elems >> LR)) || tid < (elems >> LR);
    const uint8_t* pocc = plane_occ + (size_t)c * g.nw;
    constexpr int nr = n >> LR;
    // the channel's flag words (uniform) and this thread's word within a plane
    const uint16_t* sfl = sflags + (size_t)c * g.nw * nr;
    const uint32_t fb = (uint32_t)(tid / BS);
    const uint32_t toff = fb * B + (uint32_t)(tid % BS);
    const size_t plane_elems = PAD ? g.plane_elems : ((size_t)1 << (2 * LOG2N));
    const typename Cx<R>::T* cin = inter + (size_t)c * g.nw * plane_elems;

    // comp is the Kahan compensation (float only); acci / compi the imaginary part (CPLX)
    constexpr int EI = CPLX ? E : 1;
    R acc[E], comp[sizeof(R) == 4 ? E : 1], acci[EI], compi[sizeof(R) == 4 ? EI : 1];
    comp[0] = (R)0;
    acci[0] = (R)0;
    compi[0] = (R)0;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        acc[s] = (R)0;
        if constexpr (sizeof(R) == 4) comp[s] = (R)0;
        if constexpr (CPLX) {
            acci[s] = (R)0;
            if constexpr (sizeof(R) == 4) compi[s] = (R)0;
        }
        int col, ip;
        double v = 0.0;
        if (last_slot<LOG2N, LR, BS, NT>(tid, s, col, ip)) {
            const int i = ((ip + hn) & nmask) - crop, j = (jb << LOG2BS) + col;   // image pixel
            if (!PAD || (i >= 0 && i < nimg)) {
                const double l = (double)(j - (nimg >> 1)) * g.pixel, m = (double)(i - (nimg >> 1)) * g.pixel;
                const double r2 = m * m + l * l;
                v = -r2 / (1.0 + sqrt(1.0 - r2));
            }
        }
        if constexpr (SH::NM1_LDS) nm1s[s * NT + tid] = v;
        else nm1r[s] = v;
    }
    const double w_lo = sc[c].w_lo, dw = sc[c].dw, sum_w = sc[c].sum_w, w_c0 = sc[c].w_c0;

    // the channel's plane flags, copied to LDS once (read by every plane step)
    uint8_t* ptab = reinterpret_cast<uint8_t*>(smem_raw) + SH::PTAB_OFF;
    for (int i = tid; i < g.nw; i += NT) ptab[i] = pocc[i];
    __syncthreads();
    auto next_plane = [&](int k0) {
        while (k0 < g.nw && !ptab[k0]) ++k0;
        return k0;
    };
    // the block's first column within its layout block
    const int j0 = jb << LOG2BS;
    const C* cblk = cin + (size_t)(j0 >> LOG2B) * B * n + (j0 & (B - 1));

    // planes k (in x), kn (its data in pf, loaded one plane ahead) and kn2 (its strip flags
    // in fl, loaded two planes ahead)
    int k = next_plane(0);
    int kn = k < g.nw ? next_plane(k + 1) : g.nw;
    C x[E], pf[E];
    uint32_t fl = 0;
    if (k < g.nw) {
        if (first_active) fl = sfl[(uint32_t)k * nr + fb];
        pass2_data<R, LOG2N, LR, B>(cblk + (size_t)k * plane_elems, fl, toff, pf);
        fl = (first_active && kn < g.nw) ? sfl[(uint32_t)kn * nr + fb] : 0u;
    }
    while (k < g.nw) {
        const int kn2 = kn < g.nw ? next_plane(kn + 1) : g.nw;
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = pf[m];
        if constexpr (Pass2Prefetch<R>::value) {
            if (kn < g.nw) {
                pass2_data<R, LOG2N, LR, B>(cblk + (size_t)kn * plane_elems, fl, toff, pf);
                fl = (first_active && kn2 < g.nw) ? sfl[(uint32_t)kn2 * nr + fb] : 0u;
            }
        }
        // first pass: radix E with L = 1 (no twiddles), registers to LDS
        C* la = lds0;
        if (first_active) {
            dft_small<E>(x);
            const int col = tid % BS, b = tid / BS;
            const int base = (col << LOG2N) + (b << LR);
#pragma unroll
            for (int m = 0; m < E; ++m) la[lds_pad(base + m)] = x[m];
        }
        __syncthreads();
        stockham_range<LOG2N, LR, LR, FftPlan<LOG2N, LR>::LAST_L, BS, NT>(la, tw);
        fft_last_to_regs<LOG2N, LR, BS, NT>(la, tw, x);
        double wk;
        {
#pragma clang fp contract(off)
            wk = g.wsup ? w_c0 + (double)k * dw : w_lo + ((double)k + 0.5) * dw;
        }
#pragma unroll
        for (int s = 0; s < E; ++s) {
            double cyc = wk * (SH::NM1_LDS ? nm1s[s * NT + tid] : nm1r[SH::NM1_LDS ? 0 : s]);
            cyc -= rint(cyc);
            R sn, cs;
            if constexpr (sizeof(R) == 4) {
                // hardware sin/cos of 2 pi t, t in turns (|t| <= 1/2): 1.3e-7 absolute error
                const float t = (float)cyc;
                sn = __builtin_amdgcn_sinf(t);
                cs = __builtin_amdgcn_cosf(t);
            } else {
                sincos_turn(cyc, &sn, &cs);
            }
            const R val = x[s].x * cs - x[s].y * sn;
            if constexpr (sizeof(R) == 4) {
                const R y = val - comp[s];
                const R tt = acc[s] + y;
                comp[s] = (tt - acc[s]) - y;
                acc[s] = tt;
            } else {
                acc[s] += val;
            }
            if constexpr (CPLX) {
                const R vim = x[s].x * sn + x[s].y * cs;
                if constexpr (sizeof(R) == 4) {
                    const R y = vim - compi[s];
                    const R tt = acci[s] + y;
                    compi[s] = (tt - acci[s]) - y;
                    acci[s] = tt;
                } else {
                    acci[s] += vim;
                }
            }
        }
        if constexpr (!Pass2Prefetch<R>::value) {
            if (kn < g.nw) {
                pass2_data<R, LOG2N, LR, B>(cblk + (size_t)kn * plane_elems, fl, toff, pf);
                fl = (first_active && kn2 < g.nw) ? sfl[(uint32_t)kn2 * nr + fb] : 0u;
            }
        }
        __syncthreads();
        k = kn;
        kn = kn2;
    }

    const bool scale_ok = g.unnormalized || sum_w > 0.0;
    const R inv_sw = g.unnormalized ? (R)1 : (sum_w > 0.0 ? (R)(1.0 / sum_w) : (R)0);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        int col, ip;
        if (last_slot<LOG2N, LR, BS, NT>(tid, s, col, ip)) {
            const int i = ((ip + hn) & nmask) - crop, j = (jb << LOG2BS) + col;
            if (!PAD || (i >= 0 && i < nimg)) {
                // column j of the transposed image (k_transpose makes it row-major)
                const size_t o = (size_t)c * nimg * nimg + (size_t)j * nimg + i;
                const R ti = inv_taper[i], tj = inv_taper[j];
                // the w-kernel's transform at dw (n - 1) divides the image too
                const R iw = g.wsup ? (R)(1.0 / kb_transform(dw * (SH::NM1_LDS ? nm1s[s * NT + tid]
                                                                           : nm1r[SH::NM1_LDS ? 0 : s]),
                                                             g.wsup, g.wbeta, g.wscale))
                                    : (R)1;
                const R re = scale_ok ? acc[s] * ti * tj * inv_sw * iw : (R)0;
                if constexpr (CPLX) {
                    const R im = scale_ok ? acci[s] * ti * tj * inv_sw * iw : (R)0;
                    reinterpret_cast<C*>(image)[o] = cmake<C>(re, im);
                } else {
                    image[o] = re;
                }
            }
        }
    }
}

// The stacking pass writes the image transposed, [channel][column j][row i]: a stacking block
// holds one (or a few) image columns, and written row-major its stores were 4-byte pieces of
// lines shared with 31 other blocks, which reached HBM about 8x amplified (525 MB written for
// the 67 MB of a 4096^2 image).  Column-major they are whole contiguous runs; this kernel then
// moves 64 x 64 tiles through LDS into the row-major image.  Grid (ceil(n/64), ceil(n/64), nch).
template <typename T>
__global__ void __launch_bounds__(256) k_transpose(int n, const T* __restrict__ src, T* __restrict__ dst) {
    __shared__ T tile[64][65];
    const size_t plane = (size_t)n * n * blockIdx.z;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;      // image rows i, columns j
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int j = j0 + r, i = i0 + tx;
        if (j < n && i < n) tile[r][tx] = src[plane + (size_t)j * n + i];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int i = i0 + r, j = j0 + tx;
        if (i < n && j < n) dst[plane + (size_t)i * n + j] = tile[tx][r];
    }
}

// ---------------------------------------------------------------------------------------
// Prediction (degridding): the transpose of the unnormalised imaging operator.
//
// For a real image X, y_m = sum_{a,b} G(q0+a-x_m) G(p0+b-y_m) g_k[p0+b][q0+a] with
//   g_k = the 2D transform with the - sign (phase centre N/2) of
//         X / (C(xi_i) C(xi_j)) * exp(-2 pi i w_k (n_ij - 1)),
// so that sum_ij A(z)_ij X_ij = Re sum_m z_m conj(y_m) for the imaging operator A of the
// kernels above.  The - transform is taken as the conjugate of the + transform of the
// conjugate, so the same FFT code and twiddles serve both directions.  The steps run in the
// reverse order of imaging: columns first (k_adj_cols), then rows and the degridding
// (k_adj_rows), over the same sort and the same occupied strips.

// Work-group (jb, c) = block of B image columns of channel c.  Per occupied plane: the
// conjugate of Y_k goes to LDS in bin order (image row i at position (i + N/2) mod N), one +
// transform per column, and the conjugate of the result is written for the rows of occupied
// strips in the intermediate's column-block layout (row p at p' = (p + N/2) mod N).
template <typename R, int LOG2N>
__global__ void __launch_bounds__((Shape<R, LOG2N>::NT2A))
k_adj_cols(Geom g, const Scalars* __restrict__ sc, const uint8_t* __restrict__ occ,
           const uint8_t* __restrict__ plane_occ, const R* __restrict__ image,
           const typename Cx<R>::T* __restrict__ tw, const R* __restrict__ inv_taper,
           typename Cx<R>::T* __restrict__ inter) {
    using C = typename Cx<R>::T;
    using SH = Shape<R, LOG2N>;
    constexpr int n = SH::N, nmask = n - 1, hn = n >> 1;
    constexpr int B = SH::B, BA = SH::BA, NT = SH::NT2A, LOG2B = Log2Of<B>::value_any, LR = SH::LR2A;
    constexpr int LOG2BA = Log2Of<BA>::value_any, LOG2GA = LOG2B - LOG2BA;
    constexpr int elems = BA * n;
    constexpr int PER = (elems + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* lds = reinterpret_cast<C*>(smem_raw);
    // block x = BA columns starting at image column x * BA: layout block jb, its columns col0..
    const int jb = blockIdx.x >> LOG2GA, col0 = (blockIdx.x & ((1 << LOG2GA) - 1)) << LOG2BA, c = blockIdx.y;
    const int tid = threadIdx.x;
    const uint8_t* pocc = plane_occ + (size_t)c * g.nw;
    const uint8_t* socc = occ + (size_t)c * g.nb1;
    const R* img = image + (size_t)c * g.n_img * g.n_img;

    // this thread's pixels e = tid + t * NT (column (e >> LOG2N) of the block, bin e mod N)
    R xt[PER];
    double nm1[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = tid + t * NT;
        xt[t] = (R)0;
        nm1[t] = 0.0;
        if (PER * NT == elems || e < elems) {
            const int col = e >> LOG2N, ip = e & nmask;
            const int i = ((ip + hn) & nmask) - g.crop, j = (jb << LOG2B) + col0 + col;   // image pixel
            if (i >= 0 && i < g.n_img) {       // outside the image (a padded grid): zero
                xt[t] = img[(size_t)i * g.n_img + j] * inv_taper[i] * inv_taper[j];
                const double l = (double)(j - (g.n_img >> 1)) * g.pixel, m = (double)(i - (g.n_img >> 1)) * g.pixel;
                const double r2 = m * m + l * l;
                nm1[t] = -r2 / (1.0 + sqrt(1.0 - r2));
            }
        }
    }
    const double w_lo = sc[c].w_lo, dw = sc[c].dw;
    for (int k = 0; k < g.nw; ++k) {
        if (!pocc[k]) continue;
        double wk;
        {
#pragma clang fp contract(off)
            wk = w_lo + ((double)k + 0.5) * dw;
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + t * NT;
            if (PER * NT == elems || e < elems) {
                double cyc = wk * nm1[t];
                cyc -= rint(cyc);
                R sn, cs;
                if constexpr (sizeof(R) == 4) {
                    const float tt = (float)cyc;
                    sn = __builtin_amdgcn_sinf(tt);
                    cs = __builtin_amdgcn_cosf(tt);
                } else {
                    sincos_turn(cyc, &sn, &cs);
                }
                // conj(X_t exp(-2 pi i cyc)) = X_t (cos, +sin)
                lds[lds_pad(e)] = cmake<C>(xt[t] * cs, xt[t] * sn);
            }
        }
        __syncthreads();
        fft_rows_lds<LOG2N, LR, BA, NT>(lds, tw);
        C* dst = inter + (size_t)(c * g.nw + k) * g.plane_elems + (size_t)jb * B * n + col0;
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int f = tid + t * NT;       // [p'][col] order: BA contiguous columns of each row
            if (PER * NT == elems || f < elems) {
                const int pp = f >> LOG2BA, col = f & (BA - 1);
                const int p = (pp + hn) & nmask;
                if (socc[k * g.S + (p >> g.log2H)]) {
                    const C v = lds[lds_pad((col << LOG2N) + pp)];
                    dst[(size_t)pp * B + col] = cmake<C>(v.x, -v.y);
                }
            }
        }
        __syncthreads();
    }
}

// One occupied strip (plane k of channel c, strip s): its rows of the intermediate, the row
// transform (- sign, as above) in LDS, then every record whose taps reach the strip reads
// them and adds its partial sum to its visibility.
template <typename R, int LOG2N, int WMAX>
__device__ __forceinline__ void degrid_strip(const Geom& g, int c, int k, int s, unsigned char* smem_raw,
                                             const uint32_t* __restrict__ offsets,
                                             const uint32_t* __restrict__ rec_cell,
                                             const void* __restrict__ rec,
                                             const uint32_t* __restrict__ rec_idx,
                                             const R* __restrict__ kbc,
                                             const typename Cx<R>::T* __restrict__ tw,
                                             const typename Cx<R>::T* __restrict__ inter,
                                             typename Cx<R>::T* __restrict__ vis_out, uint32_t aux) {
    using C = typename Cx<R>::T;
    using SH = Shape<R, LOG2N>;
    constexpr int n = SH::N, H = SH::H, NT = SH::NT1, nmask = n - 1, hn = n >> 1;
    constexpr int LOG2H = Log2Of<H>::value_any;
    constexpr int B = SH::B, LOG2B = Log2Of<B>::value_any;
    constexpr int elems = H * n;
    constexpr int LHB = LOG2H + LOG2B;
    C* lds = reinterpret_cast<C*>(smem_raw);
    const int tid = threadIdx.x;
    const int row0 = s * H;
    const int pp0 = (row0 + hn) & nmask;        // a strip never wraps in p' (H divides N/2)
    const C* src = inter + (size_t)(c * g.nw + k) * g.plane_elems;
    if (g.crop > 0) {      // a padded grid: the columns outside the image are zero
        for (int e = tid; e < elems; e += NT) lds[lds_pad(e)] = cmake<C>((R)0, (R)0);
        __syncthreads();
    }
    const int in_elems = H * g.n_img;
    for (int e = tid; e < in_elems; e += NT) {
        const int jb = e >> LHB, rem = e & ((1 << LHB) - 1);
        const int lr = rem >> LOG2B, col = rem & (B - 1);
        const int j = g.crop + (jb << LOG2B) + col;
        const C v = src[((size_t)jb << LOG2N) * B + (size_t)(pp0 + lr) * B + col];
        lds[lds_pad((lr << LOG2N) + ((j + hn) & nmask))] = cmake<C>(v.x, -v.y);
    }
    __syncthreads();
    fft_rows_lds<LOG2N, SH::LR1, H, NT>(lds, tw);

    const int W = g.support;
    int s_lo = (row0 - (W - 1)) >> LOG2H;
    if (s_lo < 0) s_lo = 0;
    const int bucket0 = c * g.nb1 + k * g.S;
    // a split strip: every part transforms the strip and degrids its share of the records
    uint32_t pb = offsets[(size_t)(bucket0 + s_lo) << kLogReplicas];
    uint32_t pe = offsets[(size_t)(bucket0 + s + 1) << kLogReplicas];
    const uint32_t parts = aux & 0xFFu, part = (aux >> 8) & 0xFFu;
    if (parts > 1) {
        const uint64_t len = pe - pb;
        const uint32_t b0 = pb;
        pb = b0 + (uint32_t)(len * part / parts);
        pe = b0 + (uint32_t)(len * (part + 1) / parts);
    }
    for (int sp = s_lo; sp <= s; ++sp) {
        uint32_t beg = offsets[(size_t)(bucket0 + sp) << kLogReplicas];
        uint32_t end = offsets[(size_t)(bucket0 + sp + 1) << kLogReplicas];
        beg = beg > pb ? beg : pb;
        end = end < pe ? end : pe;
        for (uint32_t r = beg + tid; r < end; r += NT) {
            int q0, p0;
            C fr, v;
            decode_record<R>(fetch_record<R>(rec_cell, rec, r), sp, LOG2H, q0, p0, fr, v);
            int b_lo = row0 - p0;
            if (b_lo < 0) b_lo = 0;
            int b_hi = row0 + H - 1 - p0;
            if (b_hi > W - 1) b_hi = W - 1;
            if (b_lo > b_hi) continue;
            R gx[WMAX];
#pragma unroll
            for (int a = 0; a < WMAX; ++a)
                if (a < W) gx[a] = kb_tap<R>(kbc, a, fr.x);
            R sr = (R)0, si = (R)0;
            for (int b = b_lo; b <= b_hi; ++b) {
                const R gy = kb_tap<R>(kbc, b, fr.y);
                const int lrow = (p0 + b - row0) << LOG2N;
                R tr = (R)0, ti = (R)0;
#pragma unroll
                for (int a = 0; a < WMAX; ++a) {
                    if (a < W) {
                        const C h = lds[lds_pad(lrow + ((q0 + a + hn) & nmask))];
                        tr += gx[a] * h.x;
                        ti -= gx[a] * h.y;      // the conjugate undoes the transform's conjugation
                    }
                }
                sr += gy * tr;
                si += gy * ti;
            }
            const uint32_t m = rec_idx[r];
            if (v.x != (R)0) si = -si;      // folded row: the transpose of gridding conj(z)
            unsafeAtomicAdd(&vis_out[m].x, sr);
            unsafeAtomicAdd(&vis_out[m].y, si);
        }
    }
}

// Persistent over the work list of occupied strips of all channels (as k_grid_rows).
template <typename R, int LOG2N, int WMAX>
__global__ void __launch_bounds__((Shape<R, LOG2N>::NT1))
k_adj_rows(Geom g, WorkList* __restrict__ wl, const uint32_t* __restrict__ list,
           const uint32_t* __restrict__ list_aux, uint32_t list_cap,
           const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ rec_cell,
           const void* __restrict__ rec, const uint32_t* __restrict__ rec_idx, const R* __restrict__ kbc,
           const typename Cx<R>::T* __restrict__ tw, const typename Cx<R>::T* __restrict__ inter,
           typename Cx<R>::T* __restrict__ vis_out) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int item;
    __shared__ uint32_t item_aux;
    uint32_t spent = 0u;        // thread 0's mask of exhausted work-list sources
    unsigned n_heavy = 0u, n_light = 0u;
    if (threadIdx.x == 0) { n_heavy = wl->n_heavy; n_light = wl->n_light; }
    while (true) {
        if (threadIdx.x == 0) {
            uint32_t x = 1u;
            item = fetch_item(wl, list, list_aux, list_cap, n_heavy, n_light, x, spent);
            item_aux = x;
        }
        __syncthreads();
        const int b = item;
        const uint32_t aux = item_aux;
        __syncthreads();
        if (b < 0) break;
        const int c = b / g.nb1, bb = b - c * g.nb1;
        const int k = bb / g.S, s = bb - k * g.S;
        degrid_strip<R, LOG2N, WMAX>(g, c, k, s, smem_raw, offsets, rec_cell, rec, rec_idx, kbc,
                                     opaque_ptr(tw), inter, vis_out, aux);
        __syncthreads();
    }
}

}  // namespace wsimg
