/*
 * fobf.h -- C ABI of the MI355X (gfx950) Fourier bilateral filter library.
 *
 * Method: "Optimized Fourier Bilateral Filtering", S. Ghosh, P. Nair,
 * K. N. Chaudhury, IEEE Signal Processing Letters 25(10), 2018.
 *
 *   bilateral filter ............. eq. (1), Gaussian kernels eq. (2)
 *   K-term cosine range kernel ... eq. (3), period 2T+1
 *   kernel error / LS fit ........ eq. (4), (5)
 *   period search, order search .. eq. (6), Algorithm 1
 *
 * Conventions shared by every entry point
 *   - Images are single-channel float32, row-major; element (y, x) of an
 *     image with leading dimension ld sits at ptr[y * ld + x].
 *   - The spatial window is the square of radius r = ceil(3 * theta)
 *     (the (6 theta + 1)^2 window of Sec. I) with separable taps
 *     g(m) = exp(-m^2 / (2 theta^2)), g(0) = 1.
 *   - Neighbours outside the image are left out of both sums of eq. (1)
 *     (equivalently, every convolved channel is zero padded).
 *   - The output is N / D literally: no clamping.  Where the cosine series
 *     of eq. (3) dips below zero D can be <= 0 and the pixel is unreliable.
 *   - Device pointers are caller-owned; the library never frees them.
 *   - Non-OK statuses leave a message for fobf_last_error() (thread-local).
 *   - fobf_fit and fobf_filter* are reentrant.  fobf_filter* only enqueue
 *     work on the given HIP stream (NULL = the null stream) and never
 *     synchronise; faults inside kernels surface at the caller's next sync.
 */
#ifndef FOBF_H
#define FOBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FOBF_OK = 0,
  FOBF_WARN_TOL = 1,   /* fit done, but its kernel error E exceeds eps; or a
                          filter ran FOBF_FP16_STAGE as FOBF_FP16X2_STAGE  */
  FOBF_EBUSY = 2,      /* serving: not finished yet / no capacity, retry    */
  FOBF_EINVAL = -1,    /* invalid argument                                  */
  FOBF_ENOMEM = -2,    /* allocation failed or request exceeds the budget   */
  FOBF_EHIP = -3,      /* a HIP runtime call failed                         */
  FOBF_EINTERNAL = -4, /* internal error                                    */
  FOBF_ECANCELED = -5, /* serving: request cancelled or server stopped      */
  FOBF_ETIMEDOUT = -6  /* serving: not admitted before its deadline         */
} fobf_status;

typedef enum {
  FOBF_FP32 = 0,        /* channels and intermediates stored in float32     */
  FOBF_FP16_STAGE = 1,  /* channels/intermediates staged in fp16, fp32 acc.
                           Error ~ 2^-9 sum|c_k| (local contrast) / (D/W).
                           Used only for series without negative lobes
                           (fobf_effective_prec); a crude series, whose
                           lobes leave D/W small, runs as FOBF_FP16X2_STAGE
                           and the call returns FOBF_WARN_TOL               */
  FOBF_BF16_STAGE = 2,  /* staged as two bf16 words (hi + lo), fp32 acc      */
  FOBF_FP16X2_STAGE = 3 /* staged as two fp16 words (hi + lo), fp32 acc:
                           float32-class accuracy on the fp16 matrix cores  */
} fobf_prec;

typedef enum {
  FOBF_ALGO_AUTO = 0,   /* library picks (tuned table, else heuristics)     */
  FOBF_ALGO_VALU = 1,   /* vector-ALU separable convolution (fp32 only)     */
  FOBF_ALGO_MFMA = 2    /* banded-Toeplitz matrix-core convolution          */
} fobf_algo;

#define FOBF_KMAX 32   /* largest order K (number of cosine terms)           */
#define FOBF_RMAX 48   /* largest spatial radius ceil(3 theta), theta <= 16 */

/* Result of a fit: the cosine series phi_hat(t) = sum_k c[k] cos(2 pi k t /
 * (2T+1)) of eq. (3).  Plain value type. */
typedef struct {
  int R;                 /* intensity range: t runs over the integers -R..R */
  int K;                 /* order (number of coefficients)                  */
  int T;                 /* period parameter; the period is 2T+1            */
  int Tmax;              /* upper end of the period scan used               */
  double sigma;          /* range std-dev (0 for fobf_fit_samples)          */
  double E;              /* kernel error E(K,T) of eq. (5) at the optimum   */
  double delta;          /* max_t |phi(t) - phi_hat(t)| over t in -R..R     */
  double c[FOBF_KMAX];   /* c[0..K-1]; entries >= K are zero                */
} fobf_coef;

/*
 * fobf_fit -- least-squares coefficients and optimal period
 *             (eq. (4)-(6), Algorithm 1).
 *
 * K >= 1 : fixed order.  Scans T = max(1, K-1) .. Tmax, solving eq. (5)
 *          exactly for each T (float64 Householder QR of the system folded
 *          onto t >= 0), and keeps the smallest E (smallest T on ties).
 *          Returns FOBF_WARN_TOL when that E exceeds eps (out is valid).
 * K == 0 : Algorithm 1: the smallest K <= FOBF_KMAX whose best period meets
 *          E <= eps; FOBF_EINVAL if none does.
 * Tmax <= 0 selects the default 4R.  Requires R >= 1, sigma > 0, eps > 0,
 * 0 <= K <= min(FOBF_KMAX, R+1).  Results are cached per (R, sigma, K,
 * eps, Tmax); thread-safe.
 */
fobf_status fobf_fit(int R, double sigma, int K, double eps, int Tmax,
                     fobf_coef* out);

/*
 * fobf_fit_warm -- the same fixed-order fit as fobf_fit (K >= 1), with the
 * period found by a local search started at T0 instead of the full scan.
 * The paper notes that E(K, T) is unimodal in T for fixed K (Sec. II, after
 * Algorithm 1).  The search walks downhill from T0 with doubling steps until
 * E rises, then narrows that bracket by golden-section steps: about 20-30
 * least-squares solves instead of Tmax - K + 2.  Measured on the Gaussian
 * kernel, E decreases strictly from about T = R/2 up to T* and increases
 * strictly from there to at least 3.4 R (R = 31 .. 1023, sigma = 0.04 R ..
 * 0.4 R, K = 2 .. 12), so any T0 in that range -- T0 = R in particular --
 * gives the scan's T*, except where E has reached the float64 floor
 * (E < 1e-12) and several periods are equally good.  Below about R/2, and
 * for K >= 11 close to 4R, E(K, T) has ripples: a start there can stop at
 * a local minimum.
 *
 * T0 <= 0 starts at T0 = R; T0 is clamped to [max(1, K-1), Tmax].  A table
 * read-out (fobf_lut_fit) gives a start near T*: fobf_fit_warm(R, sigma,
 * lut K, eps, 0, lut T, out) refines it.  Arguments and statuses otherwise
 * as fobf_fit with K >= 1 (FOBF_WARN_TOL when E > eps).  Not cached;
 * thread-safe.
 */
fobf_status fobf_fit_warm(int R, double sigma, int K, double eps, int Tmax, int T0,
                          fobf_coef* out);

/*
 * fobf_fit_period -- the least-squares coefficients of eq. (5) at one given
 * period T (no scan over T).  T = R is the fixed period [-R, R] of the
 * earlier Fourier bilateral filter the paper compares against (Sec. III,
 * Figs. 3-4); there the columns of A are orthogonal on the integers of
 * [-R, R] and c is the discrete Fourier projection of the samples.  Requires
 * R >= 1, sigma > 0, 1 <= K <= min(FOBF_KMAX, R+1), T >= max(1, K-1);
 * FOBF_EINVAL otherwise or when the columns are numerically dependent.
 * out->Tmax is set to T.  Not cached.
 */
fobf_status fobf_fit_period(int R, double sigma, int K, int T, fobf_coef* out);

/*
 * fobf_lut -- the offline table of optimal parameters (Sec. II, after
 * Algorithm 1; Fig. 2): K* and T* from Algorithm 1 at every point of a
 * (sigma, eps) grid.  At run time, (K, T) for an off-grid (sigma, eps) is
 * read by bilinear interpolation in (sigma, log(1/eps)) -- K rounded up, T
 * to the nearest integer and at least K - 1 -- and the coefficients come
 * from one least-squares solve at that (K, T).  The paper reports a loss of
 * at most 1-2 dB against the exact optimum.
 *
 * fobf_lut_create: sigmas[n_sigma] > 0 strictly increasing, eps[n_eps] > 0
 *   strictly decreasing, Tmax <= 0 = 4R.  Runs Algorithm 1 (fobf_fit with
 *   K = 0) at every grid point; FOBF_EINVAL if a point has no order up to
 *   FOBF_KMAX.  The table is owned by the caller (fobf_lut_destroy).
 * fobf_lut_get: (K*, T*) stored at grid point (i_sigma, i_eps).
 * fobf_lut_fit: coefficients for (sigma, eps) inside the grid (FOBF_EINVAL
 *   outside); FOBF_WARN_TOL when the interpolated (K, T) misses E <= eps
 *   (out is valid; fobf_fit with K = 0 gives the exact optimum).
 * fobf_lut_save / fobf_lut_load: text file round trip (load allocates).
 * A table is read-only after creation: concurrent lut_fit calls are safe.
 */
typedef struct fobf_lut fobf_lut;
fobf_status fobf_lut_create(int R, const double* sigmas, int n_sigma, const double* eps,
                            int n_eps, int Tmax, fobf_lut** out);
fobf_status fobf_lut_get(const fobf_lut* lut, int i_sigma, int i_eps, int* K, int* T);
fobf_status fobf_lut_fit(const fobf_lut* lut, double sigma, double eps, fobf_coef* out);
fobf_status fobf_lut_save(const fobf_lut* lut, const char* path);
fobf_status fobf_lut_load(const char* path, fobf_lut** out);
void fobf_lut_destroy(fobf_lut* lut);

/*
 * fobf_fit_cache_clear -- drops every cached fobf_fit result and returns how
 * many there were.  Later fobf_fit calls solve eq. (5) again.  Servers keep
 * their own device copies of coefficients they already use; those are not
 * affected.  Thread-safe; never fails.
 */
int fobf_fit_cache_clear(void);

/*
 * fobf_fit_cache_save / fobf_fit_cache_load -- keep fobf_fit's cache across
 * processes: save writes every cached (R, sigma, K, eps, Tmax) -> (T, c, E,
 * delta) entry to a text file (doubles in hexadecimal, so a round trip is
 * exact); load adds a file's entries to the cache (replacing equal keys),
 * after which fobf_fit returns them without solving eq. (5) again.  A
 * missing or malformed file gives FOBF_EINVAL and leaves the cache as it
 * was.  Thread-safe.
 */
fobf_status fobf_fit_cache_save(const char* path);
fobf_status fobf_fit_cache_load(const char* path);

/*
 * fobf_fit_samples -- the same fit for an arbitrary even range kernel given
 * by its samples b[t] = phi(t), t = 0..R (host array of R+1 doubles; the
 * kernel must be even, phi(-t) = phi(t)).  The paper notes that the LS
 * model applies to non-Gaussian kernels unchanged (Sec. I, contributions).
 * K >= 1 only; not cached.  out->sigma is set to 0.
 */
fobf_status fobf_fit_samples(int R, const double* b, int K, double eps,
                             int Tmax, fobf_coef* out);

/*
 * fobf_filter -- the K-term shiftable bilateral filter on one image.
 *
 * Computes, for every pixel i,
 *   N(i) = sum_k c_k [cos(nu k f(i)) (w*(cos(nu k f) f))(i)
 *                     + sin(nu k f(i)) (w*(sin(nu k f) f))(i)]
 *   D(i) = the same with the factor f dropped inside the convolutions,
 * nu = 2 pi / (2T+1), w = the truncated Gaussian spatial kernel, and
 * writes out(i) = N(i) / D(i).  This equals eq. (1) with phi replaced by
 * phi_hat of eq. (3) (Sec. II, first paragraph).
 *
 * d_in   device pointer, H x W floats with leading dimension ld_in.
 * d_out  device pointer, H x W floats with leading dimension ld_out; must
 *        not overlap d_in (tiles read their neighbours' halo).
 * theta  spatial std-dev, 0 < theta, ceil(3 theta) <= FOBF_RMAX.
 * K, T   order and period parameter, 1 <= K <= FOBF_KMAX, T >= 1.
 * c      host array of K doubles (copied before return).
 * prec   fobf_prec; algo fobf_algo (FOBF_ALGO_VALU supports FOBF_FP32 only).
 *        The staged modes subtract the tile-centre value m from f before
 *        rounding (exact: N - m D is accumulated, out = N'/D + m); fp16
 *        words hold magnitudes below 65504, so the fp16 modes suit images
 *        whose local contrast times the tap sum (~2.5 theta) stays below
 *        that, e.g. 8- to 12-bit intensities.
 * stream hipStream_t as void* (NULL = null stream).
 * H, W >= 1, ld >= W.  H == 0 or W == 0 is a no-op returning FOBF_OK.
 * Enqueues kernels only (no allocation, copy or memset), so the call can
 * be captured in a HIP graph; launch errors are returned, device faults
 * surface at the caller's next synchronisation.  Returns FOBF_WARN_TOL
 * (output valid) when FOBF_FP16_STAGE ran as FOBF_FP16X2_STAGE
 * (fobf_effective_prec).
 */
fobf_status fobf_filter(const float* d_in, float* d_out, int H, int W,
                        int ld_in, int ld_out, double theta, int K, int T,
                        const double* c, int prec, int algo,
                        void* hip_stream);

/*
 * fobf_effective_prec -- the precision fobf_filter, fobf_filter_ws,
 * fobf_filter_batch and the server run for the requested `prec` and the
 * cosine series (K, T, c) of eq. (3).  Every precision runs as requested
 * except FOBF_FP16_STAGE for a series whose lowest value over one period
 * (2T+1) is below -1% of its peak: D/W, the window average of the series
 * over a pixel's neighbours, then comes close to zero where the negative
 * lobes meet the image's contrast, the output N/D magnifies fp16's
 * rounding past half an intensity level, and the call runs two-word fp16
 * staging (FOBF_FP16X2_STAGE) instead.  The filter calls return
 * FOBF_WARN_TOL (output valid, message in fobf_last_error) when they do
 * so.  Host-only; returns -1 for an invalid prec, K (1..FOBF_KMAX), T (>= 1)
 * or a NULL c.
 */
int fobf_effective_prec(int prec, int K, int T, const double* c);

/*
 * fobf_filter_workspace_size / fobf_filter_ws -- the same filter (Sec. II,
 * first paragraph; outputs as fobf_filter, up to float32 summation order)
 * with a caller-provided device workspace that holds each tile's running N
 * and D instead of the LDS.  That frees the LDS for tiles of up to 512 rows,
 * so far fewer of the vertical pass's halo rows are recomputed, and lets
 * FOBF_FP32 stage each block's channels once per workgroup instead of once
 * per wave (its output is then identical to fobf_filter's, bit for bit).
 * Every precision uses it for images tall enough to give such tiles while
 * still filling the device (e.g. 2048^2 and larger at theta <= 13.5),
 * FOBF_FP32 only from radius 14 on (theta > 13/3: below, the N/D round
 * trips cost more than they save); there FOBF_FP16_STAGE also folds two
 * frequencies per pass over the tile (N and D make half the round trips;
 * same output as one at a time).  For every other case the workspace is not
 * used and fobf_filter_ws behaves exactly as fobf_filter.
 *
 * fobf_filter_workspace_size: *bytes = the workspace fobf_filter_ws needs
 *   for an H x W image at this theta and precision (0: none; about 8 bytes
 *   per pixel otherwise, the same for every precision that uses it).
 *   Host-only, no device work.
 *   Validates H, W >= 0, theta, prec and bytes != NULL (FOBF_EINVAL).
 * fobf_filter_ws: arguments as fobf_filter, plus d_work (device memory, 4-
 *   byte aligned, overlapping neither image) of work_bytes >=
 *   fobf_filter_workspace_size; FOBF_EINVAL when it is needed and missing,
 *   short, misaligned or overlapping.  The workspace needs no clearing
 *   (every tile writes its N and D before reading them); it is scratch
 *   owned by the caller, and two calls in flight at once need two
 *   workspaces.  Enqueues kernels only (capturable), as fobf_filter.
 */
fobf_status fobf_filter_workspace_size(int H, int W, double theta, int prec, size_t* bytes);
fobf_status fobf_filter_ws(const float* d_in, float* d_out, int H, int W, int ld_in,
                           int ld_out, double theta, int K, int T, const double* c,
                           int prec, int algo, void* d_work, size_t work_bytes,
                           void* hip_stream);

/*
 * fobf_filter_ws_static -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): fobf_filter_ws with its workspace taken from a device array
 * the library holds instead of a caller buffer.  Arguments, validation,
 * outputs and statuses are those of fobf_filter_ws (bit-identical output);
 * the call allocates nothing and enqueues kernels only.
 *
 * The array holds FOBF_STATIC_SCRATCH_BYTES (128 MiB: N and D of one
 * 4096 x 4096 image); an image whose fobf_filter_workspace_size exceeds it
 * is rejected with FOBF_EINVAL before any device work.  Each GPU holds its
 * own copy from the first call on it (made with that GPU current; the
 * stream must belong to the calling thread's current device) until the
 * process ends.  Every call on one GPU shares that GPU's copy and leaves
 * the last call's partial sums in it: calls whose work overlaps on one GPU
 * (two streams, or two threads) race and must be ordered by the caller.
 * Nothing in it needs clearing: each tile writes its N and D before reading
 * them.
 */
#define FOBF_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
fobf_status fobf_filter_ws_static(const float* d_in, float* d_out, int H, int W, int ld_in,
                                  int ld_out, double theta, int K, int T, const double* c,
                                  int prec, int algo, void* hip_stream);

/* One image of a batch (all pointers device pointers, caller-owned). */
typedef struct {
  const float* d_in;
  float* d_out;
  int H, W, ld_in, ld_out;
  double theta;
  int K, T;
  int prec;              /* fobf_prec                                       */
  double c[FOBF_KMAX];
} fobf_job;

/*
 * fobf_filter_batch -- filter n independent images of different sizes and
 * parameters with persistent launches: every workgroup pulls output tiles
 * from a shared queue that spans all jobs (work stealing), so small and
 * large images, and different radii and orders, share the machine.  All
 * jobs of one precision and radius class (r <= 24, 24 < r <= 32, or
 * 32 < r <= 48) go
 * into ONE launch; a batch of one precision and class is one launch.
 *
 * jobs      host array of n jobs (read before return; the job table is
 *           copied through a library-owned pinned buffer).
 * d_work    device workspace of at least fobf_batch_workspace_size(n)
 *           bytes, 256-byte aligned, caller-owned, not used by another
 *           call until this call's work on the stream has finished.
 * Same rules per job as fobf_filter (algorithm: matrix cores; a job's
 * FOBF_FP16_STAGE may run as FOBF_FP16X2_STAGE, fobf_effective_prec, and
 * the call then returns FOBF_WARN_TOL naming the last such job).  Jobs with
 * H == 0 or W == 0 are skipped; n == 0 is a no-op.  Unlike fobf_filter
 * (kernels only, capturable in a HIP graph), a batch call copies its job
 * table from library-owned pinned memory, so it is not meant for graph
 * capture.
 */
size_t fobf_batch_workspace_size(int n);
fobf_status fobf_filter_batch(const fobf_job* jobs, int n, void* d_work,
                              size_t work_bytes, void* hip_stream);

/* ------------------------------------------------------------------------
 * Tile-shape autotuner.
 *
 * fobf_filter (FOBF_ALGO_AUTO) and fobf_filter_batch read a process-wide
 * table that picks, per precision and radius class dv = ceil((16 + 2r)/16),
 * the algorithm (float32: matrix cores or vector ALU) and the tile height.
 * fobf_autotune times every candidate for one precision on an H x W image
 * of order K on the device (it allocates two temporary H x W buffers and
 * synchronises `hip_stream`) and records the fastest; until then built-in
 * defaults apply.  The table can be saved to and loaded from a text file.
 * The table's height is an upper bound: an image (or a batch launch class)
 * with fewer than four rounds of tiles per workgroup slot of the device
 * runs shorter tiles where that shortens rounds x tile chain (small images
 * are latency-bound, not throughput-bound).  Tune on images of the size
 * the table is meant for (2048^2 and up fill the device at the default).
 * ---------------------------------------------------------------------- */
fobf_status fobf_autotune(int prec, int H, int W, int K, void* hip_stream);
fobf_status fobf_tune_save(const char* path);
fobf_status fobf_tune_load(const char* path);
fobf_status fobf_tune_reset(void);
/* The choice the table makes for (prec, theta): *algo is a fobf_algo,
 * *nblk the tile height in 16-row blocks. */
fobf_status fobf_tune_get(int prec, double theta, int* algo, int* nblk);

/* ------------------------------------------------------------------------
 * Serving: continuous batching.
 *
 * Requests (host images) may be submitted from any thread at any time.  A
 * scheduler thread admits them while their device memory fits the HBM
 * budget, fits (or looks up) their coefficients in a device-resident cache
 * keyed by (R, sigma, K), copies them in on a copy stream and launches
 * their tiles; requests that arrive while others run are admitted as
 * memory frees up, and their work overlaps on the device.  Completion is
 * reported by fobf_serve_poll.
 * ---------------------------------------------------------------------- */
typedef struct fobf_server fobf_server;

typedef struct {
  size_t hbm_budget_bytes;  /* device bytes for in-flight requests (>0)    */
  int max_inflight;         /* requests in flight at once (>=1)            */
  int max_batch;            /* requests merged into one launch (>=1)       */
  int R;                    /* intensity range of the images (>=1)         */
  double eps;               /* tolerance passed to fobf_fit (>0)           */
} fobf_serve_cfg;

typedef struct {
  const float* h_in;        /* host image H x W, row-major; read while the */
                            /* request is in flight                        */
  float* h_out;             /* host output H x W; alive until polled done  */
  int H, W;
  int ld_in, ld_out;        /* host leading dimensions (0 = W)             */
  double theta, sigma;
  int K;                    /* order (>=1)                                 */
  int prec;                 /* fobf_prec                                   */
  double deadline_s;        /* admit within this many seconds of submit,   */
                            /* else FOBF_ETIMEDOUT (0 = no deadline, >= 0) */
} fobf_request;

typedef struct {
  fobf_status status;       /* FOBF_EBUSY while pending                    */
  double t_submit, t_admit, t_start, t_done;   /* seconds, monotonic clock */
  int T;                    /* fitted period used                          */
  int prec;                 /* precision the request ran in (see           */
                            /* fobf_effective_prec)                        */
} fobf_result;

fobf_status fobf_serve_create(const fobf_serve_cfg* cfg, fobf_server** out);
fobf_status fobf_serve_submit(fobf_server* s, const fobf_request* req,
                              uint64_t* ticket);
/* wait != 0 blocks until the request is done.  Returns the request's final
 * status (copied into *res too) or FOBF_EBUSY while it is pending.  Once a
 * final status has been returned the ticket is released: polling it again
 * gives FOBF_EINVAL.  Thread-safe. */
fobf_status fobf_serve_poll(fobf_server* s, uint64_t ticket, int wait,
                            fobf_result* res);
/* Cancels a request that is still queued (not yet admitted to the device):
 * it completes at once with FOBF_ECANCELED (poll it to release the ticket)
 * and returns FOBF_OK.  FOBF_EBUSY when the request is already on the device
 * (it completes normally), FOBF_EINVAL for an unknown ticket or a request
 * that has completed.  Cancelled and timed-out requests count as completed
 * and failed in the statistics.  Thread-safe. */
fobf_status fobf_serve_cancel(fobf_server* s, uint64_t ticket);
/* Requests still queued when the server is destroyed complete with
 * FOBF_ECANCELED; work already on the device finishes first.  Tickets are
 * invalid afterwards.  No other call on the same server may be running
 * (a blocking poll must have returned) or start once destroy is called. */
fobf_status fobf_serve_destroy(fobf_server* s);

typedef struct {
  uint64_t submitted, completed, failed, batches;
  size_t peak_bytes_inflight;   /* never exceeds cfg.hbm_budget_bytes      */
  int peak_inflight;            /* never exceeds cfg.max_inflight          */
  int coef_entries;             /* distinct (R, sigma, K) fits on device   */
} fobf_serve_stats;
fobf_status fobf_serve_get_stats(fobf_server* s, fobf_serve_stats* out);

/* Test hook: the next `count` device submissions of this server report a
 * HIP error without launching anything (fault injection from the host). */
fobf_status fobf_serve_inject_fault(fobf_server* s, int count);

/* ---- debug-check build ------------------------------------------------
 * libfobf_check.so is the same library compiled with FOBF_CHECKS=1: every
 * kernel first fills its LDS allocation with all-ones words (NaN in
 * float32, fp16 and bf16), so a read of LDS the kernel never wrote reaches
 * the output as NaN, and checks its indices while it runs, recording each
 * kind of violation as a bit in one device word instead of trapping:
 *   FOBF_CHECK_LDS     LDS access outside the launch's dynamic allocation
 *   FOBF_CHECK_IMAGE   image read outside the image (unclamped paths)
 *   FOBF_CHECK_HALO_H  horizontal pass: a non-zero tap on a column outside
 *                      the output column's window, or outside the staged
 *                      columns of the block
 *   FOBF_CHECK_HALO_V  vertical pass: a non-zero tap on a row outside the
 *                      output row's window
 *   FOBF_CHECK_RING    vertical pass: a ring slot holding another block
 *                      than the one its taps are for
 *   FOBF_CHECK_WS      workspace access outside the caller's workspace
 *   FOBF_CHECK_OUT     output write outside the image or its pitch
 *   FOBF_CHECK_TILE    batch: a tile index outside its job
 *   FOBF_CHECK_STAGE   staging item outside its block row
 * The release library computes the same outputs (the checks only read). */
#define FOBF_CHECK_LDS 0x001u
#define FOBF_CHECK_IMAGE 0x002u
#define FOBF_CHECK_HALO_H 0x004u
#define FOBF_CHECK_HALO_V 0x008u
#define FOBF_CHECK_RING 0x010u
#define FOBF_CHECK_WS 0x020u
#define FOBF_CHECK_OUT 0x040u
#define FOBF_CHECK_TILE 0x080u
#define FOBF_CHECK_STAGE 0x100u

/* Waits for the device to finish all work, then returns in *bits the
 * violations recorded on the current device since the last call and
 * clears them.  FOBF_EINVAL from the release library (built without
 * checks) or when bits is NULL; FOBF_EHIP when the device cannot be read.
 * For tests and debugging: it synchronises the whole device. */
fobf_status fobf_check_take(unsigned int* bits);

/* Thread-local message for the last non-OK status of this thread. */
const char* fobf_last_error(void);

/* Library version (major * 10000 + minor * 100 + patch). */
int fobf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FOBF_H */
