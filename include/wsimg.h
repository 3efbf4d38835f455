/*
 * wsimg.h -- C ABI of the w-stacking dirty imager for AMD MI355X (gfx950).
 *
 * The library turns visibilities into a dirty image with the w-stacking method
 * of Sec. 2 of the paper: visibilities are sorted into grid strips, convolved
 * onto the nearest of Nw w-planes with a separable Kaiser-Bessel kernel (Eq. 3),
 * each plane is 2D Fourier transformed, multiplied by its w-term phase and the
 * planes are summed (Eq. 2: a per-plane w-phase, then a sum over planes), and the
 * result is divided by the kernel's Fourier transform and by the sum of weights.
 *
 * Conventions (every entry point):
 *  - All calls return a wsimg_status; 0 is success, negative values are errors.
 *    No C++ exception crosses this boundary.  wsimg_last_error() returns a
 *    thread-local text describing the most recent error of the calling thread.
 *  - Array arguments marked "device" are device pointers on the GPU the plan was
 *    created on; the caller owns them and they must stay valid until the work
 *    enqueued on the plan's stream has completed.  The plan owns its scratch.
 *  - Work is enqueued on the plan's HIP stream and returns without waiting,
 *    except where a stats pointer is given (then the call waits for the stream).
 *  - Counts are int64_t (the paper's I/O section notes the 32-bit count limit of
 *    the MPI read calls; no count here is 32-bit).
 *  - A plan is not thread-safe; separate plans are independent.
 *  - wsimg_image, wsimg_image_batch, wsimg_predict and wsimg_grid may be captured into a HIP
 *    graph (stream capture of the plan's stream) when stats is NULL: under capture they make
 *    no host wait, record no timing events, and read the channel table from a pinned buffer
 *    that only captured calls write.  A replay recomputes the outputs from the current
 *    contents of the inputs.  One captured call per plan at a time: capturing another call
 *    on the same plan rewrites the table the earlier graph reads.
 *
 * Geometry (Sec. 2, Eq. 1): u, v, w are the baseline coordinates in wavelengths,
 * (u, v, w) = uvw_m * freq_hz / c with c = 299792458 m/s.  The image is n x n,
 * row-major; pixel (i, j) has direction cosines l = (j - n/2) * pixel_rad and
 * m = (i - n/2) * pixel_rad.  The grid is n x n cells of size 1/(n * pixel_rad)
 * wavelengths, with no padding (the paper sizes its grid as the image: an
 * 8192^2 grid of 32 w-planes is 32 GB, Sec. 4.2.1).
 */
#ifndef WSIMG_H
#define WSIMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WSIMG_OK = 0,
    WSIMG_E_INVALID = -1,      /* an argument is out of range or a pointer is NULL        */
    WSIMG_E_NOMEM = -2,        /* device or host allocation failed                        */
    WSIMG_E_HIP = -3,          /* a HIP runtime call or a kernel launch failed            */
    WSIMG_E_EMPTY = -4,        /* the kept visibilities have zero total weight           */
    WSIMG_E_CAPACITY = -5,     /* n_vis exceeds the plan's max_vis                        */
    WSIMG_E_UNSUPPORTED = -6   /* valid parameters this build does not implement          */
} wsimg_status;

typedef enum {
    WSIMG_F32 = 1,   /* vis complex64, weights float32, grid/FFT/stacking float32 (Kahan
                        sum over planes); coordinates and the w-phase argument in float64 */
    WSIMG_F64 = 2    /* vis complex128, weights float64, everything float64              */
} wsimg_precision;

/* wsimg_params.flags */
#define WSIMG_FIXED_WRANGE 0x1u   /* use w_lo/w_hi below instead of the data's range     */
#define WSIMG_UNNORMALIZED 0x2u   /* wsimg_image does not divide by the sum of weights:
                                     the image is then A(W V), the imaging operator that
                                     wsimg_predict is the transpose of                    */
#define WSIMG_PAD2 0x8u           /* a grid of twice the image side (n <= 4096): the image is
                                     the central n x n of the transformed 2n x 2n grid, the
                                     cell size is 1/(2 n pixel_rad) and the taper is taken
                                     at xi = (j - n/2) / (2n), so the edge amplification of
                                     the taper division drops from C(0)^2/C(1/2)^2 to
                                     C(0)^2/C(1/4)^2 (about 6 for W = 7).  wsimg_grid then
                                     writes [n_wplanes][2n][2n]                          */
#define WSIMG_COMPLEX_OUT 0x10u    /* wsimg_image / wsimg_image_batch write the complex image
                                     S / (sum W * C(xi_j) C(xi_i)), interleaved (re, im) of
                                     the plan's real type per pixel ([n][n][2]), instead of
                                     its real part (the paper's dirty image is real, Sec. 4;
                                     the imaginary part is the image of the anti-Hermitian
                                     part of the data).  Not for wsimg_predict            */
#define WSIMG_FOLD_W 0x4u         /* w-folding: a row with w < 0 is taken as its conjugate
                                     partner (-u, -v, -w, conj V) (equal for a real sky),
                                     so the planes span |w| only; the real image is the same
                                     sum with half the w range per plane                  */

typedef struct {
    int32_t n;          /* image side = grid side: a power of two, 16..8192 (16384 is
                           accepted as valid and reported WSIMG_E_UNSUPPORTED)           */
    int32_t n_wplanes;  /* Nw >= 1, <= 4096                                                */
    int32_t support;    /* Kaiser-Bessel support W in cells: odd, 3..15                    */
    int32_t precision;  /* wsimg_precision                                                 */
    double pixel_rad;   /* pixel size dl > 0; every pixel must satisfy l^2 + m^2 < 1      */
    double beta;        /* Kaiser-Bessel shape; <= 0 selects 2.34 * support                */
    double w_lo, w_hi;  /* plane range in wavelengths when WSIMG_FIXED_WRANGE is set       */
    uint32_t flags;
    uint32_t w_support; /* 0: each visibility goes to its nearest w-plane (Sec. 2).  Odd 3..15
                           and below n_wplanes: the w-kernel across planes, Eq. 3's kernel with
                           its w argument: a Kaiser-Bessel kernel of this support along w
                           (shape 2.34 * w_support) spreads each visibility over that many
                           neighbouring planes; the planes are spaced
                           dw = (w_hi - w_lo) / (n_wplanes - w_support) with centres
                           w_lo + (k - (w_support - 1)/2) dw, and the image is also divided by
                           the w-kernel's Fourier transform at dw (n_ij - 1).  Not for
                           wsimg_predict.                                                     */
} wsimg_params;

typedef struct {
    int64_t n_in;       /* rows passed in                                                  */
    int64_t n_gridded;  /* rows kept: finite uvw and weight, all W x W taps on the grid    */
    int64_t n_dropped;  /* n_in - n_gridded                                                */
    double sum_w;       /* sum of the kept weights (the image is divided by it)           */
    double w_lo, w_hi;  /* plane range used                                                */
    int64_t n_strips_occupied;  /* (w-plane, row strip) pairs holding at least one tap: only
                                   these strips are transformed and stored between the passes */
    int64_t n_planes_occupied;  /* w-planes holding at least one kept row                      */
} wsimg_stats;

typedef struct {
    int32_t n, n_wplanes, support, precision;
    int32_t strip_rows;      /* grid rows per gridding work-group                          */
    int32_t col_block;       /* image columns per block of the row-transformed planes     */
    int64_t n_buckets;       /* sort buckets: n_wplanes * n_grid / strip_rows              */
    int64_t max_vis;
    int64_t device_bytes;    /* device memory the plan holds (or would hold)               */
    int64_t max_channels;    /* channels one wsimg_image_batch call may image              */
    int64_t n_grid;          /* grid side: n, or 2n with WSIMG_PAD2                        */
    int32_t grid_threads;    /* threads of a gridding (+ row transform) work-group         */
    int32_t stack_threads;   /* threads of a stacking (column transform) work-group        */
    int32_t stack_cols;      /* image columns per stacking work-group                      */
    int32_t stack_radix;     /* base radix of the stacking pass's column transform         */
    int64_t lds_grid_bytes;  /* dynamic LDS of a gridding work-group                       */
    int64_t lds_stack_bytes; /* dynamic LDS of a stacking work-group                       */
    int64_t record_bytes;    /* bytes of one sorted visibility record                      */
    int64_t row_capacity;    /* entries of each row-indexed scratch buffer: max_vis plus a
                                slack, so a read one entry past the last row stays inside  */
    int64_t list_capacity;   /* entries of the gridding work list                          */
} wsimg_plan_info;

#define WSIMG_N_KERNELS 8
typedef struct {
    int64_t calls;                     /* wsimg_image/wsimg_grid calls timed since enabling   */
    double ms[WSIMG_N_KERNELS];        /* summed device time of each kernel stage             */
    double ms_total;                   /* summed time from the first to the last stage         */
} wsimg_timing;

typedef struct wsimg_plan wsimg_plan;

/*
 * Create a plan for one imaging geometry on the current HIP device.
 *  out       : receives the plan (set to NULL on error).
 *  p         : parameters, copied; validated on the host before any HIP call.
 *  max_vis   : largest n_vis a call may pass, 0 .. 4294967294; scratch is sized from it.
 *  hip_stream: hipStream_t the plan's work is enqueued on (NULL = default stream).
 * Errors: WSIMG_E_INVALID (parameters), WSIMG_E_UNSUPPORTED (n = 16384),
 *         WSIMG_E_NOMEM (device memory), WSIMG_E_HIP.
 */
wsimg_status wsimg_plan_create(wsimg_plan **out, const wsimg_params *p, int64_t max_vis,
                               void *hip_stream);

/*
 * A plan that images up to max_channels channels (frequencies) of one geometry in one call
 * (wsimg_image_batch).  Every channel has its own w-plane range, planes and image; the
 * channels share the launches: each stage covers all channels of the call, and the gridding
 * work list spans the occupied strips of every channel, so many small channels fill the GPU
 * the way one large one does.
 *  max_vis      : largest total row count of a call (all channels), 0 .. 4294967294.
 *  max_channels : 1 .. 65535.  The plan's device scratch grows with it: the row-transformed
 *                 planes take max_channels * n_wplanes * n * n complex elements, the sort
 *                 counters 256 bytes per (channel, plane, strip).
 * Errors: as wsimg_plan_create; WSIMG_E_UNSUPPORTED when max_channels * n_wplanes * strips
 *         exceeds 2^25 sort buckets.
 */
wsimg_status wsimg_plan_create_batch(wsimg_plan **out, const wsimg_params *p, int64_t max_vis,
                                     int32_t max_channels, void *hip_stream);

/* Release a plan and its device memory (waits for its stream).  NULL is a no-op. */
wsimg_status wsimg_plan_destroy(wsimg_plan *plan);

/* Switch the stream later calls enqueue on. */
wsimg_status wsimg_plan_set_stream(wsimg_plan *plan, void *hip_stream);

/* Geometry and memory of a plan. */
wsimg_status wsimg_plan_get_info(const wsimg_plan *plan, wsimg_plan_info *info);

/*
 * What wsimg_plan_create_batch(p, max_vis, max_channels) would build, without building it:
 * the same checks of the parameters, then the geometry, work-group shapes and the device
 * bytes the plan would hold (every scratch allocation summed), in *info.  Host arithmetic
 * only: no HIP call, no GPU needed, nothing allocated; a caller can size its memory budget
 * (or pick max_vis / max_channels to fit it) before creating a plan.
 * Errors: as wsimg_plan_create_batch apart from WSIMG_E_NOMEM and WSIMG_E_HIP;
 *         WSIMG_E_INVALID when info is NULL.
 */
wsimg_status wsimg_plan_query(const wsimg_params *p, int64_t max_vis, int32_t max_channels,
                              wsimg_plan_info *info);

/*
 * The dirty image (Sec. 2: Eqs. 1-3, then the per-plane w-phase and the sum over planes):
 *   D(i,j) = Re sum_k P_k(i,j) exp(+2 pi i w_k (n_ij - 1)) / (sum W * C(xi_j) C(xi_i))
 * where P_k is the 2D transform (exp(+2 pi i ...), phase centre at n/2) of plane k of the
 * Kaiser-Bessel grid, w_k the plane centre, n_ij = sqrt(1 - l^2 - m^2) and C the kernel's
 * Fourier transform at xi = (j - n/2)/n.
 *  n_vis     : rows, 0 .. max_vis.
 *  uvw_m     : device, [n_vis][3] float64 row-major, metres.
 *  vis       : device, [n_vis] interleaved complex (float2 for F32, double2 for F64).
 *  weights   : device, [n_vis] float (F32) / double (F64); natural weighting (Sec. 4.2.1).
 *  freq_hz   : > 0, finite.
 *  image_out : device, [n][n] float (F32) / double (F64), row-major; fully overwritten.
 *  stats     : NULL, or receives the counters; non-NULL makes the call wait for the stream.
 * Rows whose uvw or weight is not finite, or whose W x W taps leave the grid, are dropped
 * and counted.  Planes span [w_lo, w_hi] of the kept rows with positive weight (or the
 * fixed range); a row goes to plane clamp(floor((w - w_lo)/dw), 0, Nw-1).
 * If the kept weights sum to zero the image is all zeros; with stats the call then
 * returns WSIMG_E_EMPTY.
 * Errors: WSIMG_E_INVALID, WSIMG_E_CAPACITY, WSIMG_E_HIP, WSIMG_E_EMPTY.
 */
wsimg_status wsimg_image(wsimg_plan *plan, int64_t n_vis, const double *uvw_m,
                         const void *vis, const void *weights, double freq_hz,
                         void *image_out, wsimg_stats *stats);

/*
 * Dirty images of n_channels channels, each exactly as wsimg_image would make it from that
 * channel's rows and frequency (the many frequency planes of the abstract and conclusions,
 * imaged one channel at a time by Eqs. 1-3).
 *  n_channels : 1 .. the plan's max_channels.
 *  row_counts : host, [n_channels]; channel c owns rows [sum of the counts before c,
 *               that sum + row_counts[c]) of the inputs; the total is at most max_vis.
 *  uvw_m, vis, weights : device, the rows of all channels, channel after channel, laid out
 *               as in wsimg_image.
 *  freqs_hz   : host, [n_channels], each > 0 and finite.
 *  images_out : device, [n_channels][n][n] of the plan's real type; fully overwritten.
 *  stats      : NULL, or host [n_channels] receiving each channel's counters (the call then
 *               waits for the stream).
 * The host arrays are read before the call returns.  A channel whose kept weights sum to zero
 * gets an all-zero image; with stats the call then returns WSIMG_E_EMPTY after writing every
 * channel's image and counters.
 * Errors: WSIMG_E_INVALID, WSIMG_E_CAPACITY, WSIMG_E_HIP, WSIMG_E_EMPTY.
 */
wsimg_status wsimg_image_batch(wsimg_plan *plan, int32_t n_channels, const int64_t *row_counts,
                               const double *uvw_m, const void *vis, const void *weights,
                               const double *freqs_hz, void *images_out, wsimg_stats *stats);

/*
 * Prediction (degridding): the transpose of the imaging operator, image -> visibilities.
 * With A the unnormalised imaging map of wsimg_image (WSIMG_UNNORMALIZED, gridding z_m =
 * W_m V_m), this computes y = A^T X for a real image X:
 *   Y_k = X / (C(xi_i) C(xi_j)) * exp(-2 pi i w_k (n_ij - 1)),
 *   g_k[p][q] = sum_{i,j} Y_k(i,j) exp(-2 pi i [(q-N/2)(j-N/2) + (p-N/2)(i-N/2)] / N),
 *   y_m = sum_{a,b} G(q0+a-x_m) G(p0+b-y_m) g_{k_m}[p0+b][q0+a],
 * so that sum_ij A(z)_ij X_ij = Re sum_m z_m conj(y_m) for every z.  It is the forward model
 * (Eq. 1 with the w-stacking approximation) that a data-fidelity loss differentiates through.
 *  uvw_m, freq_hz : as wsimg_image.
 *  weights   : device, [n_vis]; they only decide which rows are kept (finite) and the plane
 *              range (rows with positive weight), exactly as in wsimg_image; they do not
 *              scale the prediction.  Use WSIMG_FIXED_WRANGE to pin the planes.
 *  image_in  : device, [n][n] float (F32) / double (F64), row-major.
 *  vis_out   : device, [n_vis] interleaved complex of the plan's precision; fully
 *              overwritten (dropped rows get 0).
 *  stats     : as wsimg_image (no WSIMG_E_EMPTY: a prediction needs no weights).
 * Errors: WSIMG_E_INVALID, WSIMG_E_CAPACITY, WSIMG_E_HIP.
 */
wsimg_status wsimg_predict(wsimg_plan *plan, int64_t n_vis, const double *uvw_m, const void *weights,
                           double freq_hz, const void *image_in, void *vis_out, wsimg_stats *stats);

/*
 * The gridding step alone (Eq. 3 with the separable kernel, nearest w-plane):
 *   grid_out[k][p][q] = sum over kept rows of plane k of W_m V_m G(q - x_m) G(p - y_m)
 * where x = u / du + n/2, y = v / du + n/2 and du = 1/(n * pixel_rad).
 *  grid_out : device, [n_wplanes][n][n] interleaved complex of the plan's precision;
 *             fully overwritten.  Other arguments as wsimg_image.
 * Errors: as wsimg_image.
 */
wsimg_status wsimg_grid(wsimg_plan *plan, int64_t n_vis, const double *uvw_m,
                        const void *vis, const void *weights, double freq_hz,
                        void *grid_out, wsimg_stats *stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): wsimg_image without a plan.  Every scratch buffer
 * of the call (sort counters and records, the row-transformed planes, the tables) is carved
 * from one static device array of WSIMG_NOALLOC_SCRATCH_BYTES that the library's code object
 * holds on each GPU it runs on, from load to process end; the call makes no hipMalloc,
 * hipFree or other allocating call.  The caller still passes the inputs and the output.
 *  p        : parameters as for wsimg_plan_create (checked the same way).
 *  n_vis .. image_out : as wsimg_image; hip_stream: the stream the work is enqueued on.
 *  stats    : as wsimg_image (non-NULL waits for the stream).
 * The scratch a call needs grows with n, n_wplanes and n_vis (wsimg_plan_query's
 * device_bytes for max_vis = n_vis, plus alignment); a call that needs more than the array
 * holds returns WSIMG_E_CAPACITY before any device work (host arithmetic only).  Heavy
 * strips are not split across work-groups here (split-strip slots would have to stay zero
 * between calls), so one very dense strip can make this call slower than wsimg_image.
 * The kernel tables (twiddles, taper, kernel polynomials) are uploaded when the geometry
 * differs from the previous call's on that device; that upload waits for the stream.
 * All calls on one GPU share its array and the array keeps the last call's contents: calls
 * that overlap on one GPU (two streams, or a call before the previous one's work has
 * finished on another stream) race and give wrong images; host threads are serialised.
 * Errors: as wsimg_image; WSIMG_E_CAPACITY also for a scratch need beyond the array.
 */
#define WSIMG_NOALLOC_SCRATCH_BYTES (64u << 20)
wsimg_status wsimg_image_noalloc(const wsimg_params *p, int64_t n_vis, const double *uvw_m,
                                 const void *vis, const void *weights, double freq_hz,
                                 void *image_out, void *hip_stream, wsimg_stats *stats);

/* Per-stage device timing with HIP events on the plan's stream (enable != 0 turns it on and
 * clears the totals).  wsimg_read_timing waits for the stream and returns the totals. */
wsimg_status wsimg_set_timing(wsimg_plan *plan, int32_t enable);
wsimg_status wsimg_read_timing(wsimg_plan *plan, wsimg_timing *out);
const char *wsimg_stage_name(int32_t stage);   /* NULL when out of range */

const char *wsimg_status_string(wsimg_status s);
const char *wsimg_last_error(void);
int32_t wsimg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WSIMG_H */
