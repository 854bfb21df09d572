/*
 * libttsvd -- TT-SVD of large dense tensors on one AMD Instinct MI355X.
 *
 * C ABI.  All entry points take plain pointers and sizes, never throw, and
 * return an int status (TTSVD_OK or a negative TTSVD_E* code).  On error,
 * ttsvd_last_error() returns a message for the calling thread.  Arguments are
 * validated before anything is launched.
 *
 * Method: the optimized TSQR TT-SVD (Algorithm 2 of Roehrig-Zoellner, Thies,
 * Basermann, "Performance of the low-rank tensor-train SVD (TT-SVD) for large
 * dense tensors on modern multi-core CPUs", arXiv 2102.00104).
 *
 * Layout (Sec. 3.1.2, "Memory layout"): every matrix is column-major, and a
 * tensor X in R^{n_1 x ... x n_d} is stored in Fortran order (i_1 fastest),
 * so the unfolding ((n_1...n_{j-1}) x (n_j r_j)) of the work tensor is a plain
 * column-major matrix.  Devices pointers are HIP device memory of the current
 * device; streams are HIP streams (NULL = the legacy default stream).
 *
 * Data types: TTSVD_F64 is the paper's precision.  TTSVD_F32 and TTSVD_BF16
 * store the data in that type, accumulate block-local products in FP32 and
 * keep the triangular factors and the small SVD in FP64.
 */
#ifndef TTSVD_H
#define TTSVD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTSVD_MAX_D 64

/* Element type of tensors and work matrices. */
typedef enum ttsvd_dtype {
    TTSVD_F64 = 0,
    TTSVD_F32 = 1,
    TTSVD_BF16 = 2
} ttsvd_dtype;

/* Status codes. */
enum {
    TTSVD_OK = 0,
    TTSVD_EINVAL = -1,       /* invalid argument (sizes, strides, pointers) */
    TTSVD_ENOMEM = -2,       /* device or host allocation failed */
    TTSVD_EHIP = -3,         /* HIP runtime error (also asynchronous ones) */
    TTSVD_ENONFINITE = -4,   /* a triangular factor is not finite (NaN/Inf input) */
    TTSVD_EUNSUPPORTED = -5  /* unsupported dtype or size */
};

/*
 * ttsvd_tsqr_r -- triangular factor of a Q-less tall-skinny QR.
 *
 * Defined by the QR decomposition W = QR (Sec. 2.1.1) as computed by the
 * rank-preserving Q-less TSQR of Sec. 3.2 (Householder reflections with the
 * eps_FP safeguard of Algorithm 6, a flat reduction per row block and a
 * reduction tree over the blocks' triangular factors).
 *
 *   W      device, rows x cols, column-major, leading dimension ld >= rows,
 *          element type dtype.  Read only; never written.
 *   R      device, FP64, cols x cols, column-major, leading dimension
 *          ldr >= cols.  On return the upper triangle holds R with
 *          R^T R = W^T W (up to rounding) and the strict lower triangle is 0.
 *          If rows < cols only the first rows rows of R are significant;
 *          rows rows..cols-1 are set to 0.  Row signs are unspecified.
 *   ws     device workspace of ws_bytes bytes (see ttsvd_tsqr_workspace_size),
 *          or NULL: the library then takes a block of its device buffer
 *          cache and returns it to the cache from a host callback enqueued on
 *          `stream` after the launches (the call stays asynchronous).
 *   stream HIP stream; the call is asynchronous with respect to the host.
 *
 * Errors: TTSVD_EINVAL for rows < 1, cols < 1, ld < rows, ldr < cols, NULL
 * W or R, or a too small ws; TTSVD_EUNSUPPORTED for an unknown dtype;
 * TTSVD_EHIP for launch failures.
 */
int ttsvd_tsqr_r(const void *W, int dtype, int64_t rows, int64_t cols,
                 int64_t ld, double *R, int64_t ldr, void *ws,
                 size_t ws_bytes, hipStream_t stream);

/* Bytes of device workspace ttsvd_tsqr_r needs for this shape. */
size_t ttsvd_tsqr_workspace_size(int dtype, int64_t rows, int64_t cols);

/*
 * ttsvd_tsqr_r_noalloc -- ttsvd_tsqr_r without any device allocation.
 *
 * For callers that cannot allocate device memory during the call (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and result as ttsvd_tsqr_r, minus the
 * workspace: the triangular factors of the reduction tree live in one fixed
 * device array of TTSVD_NOALLOC_SCRATCH_BYTES bytes inside the library (one
 * copy per GPU, held until the process ends; its address is looked up once
 * per device).  The call makes no hipMalloc, hipFree or other allocating
 * call; W is read only and R is written as by ttsvd_tsqr_r.
 *
 * All calls on one GPU share that array, whose contents persist from call
 * to call (nothing in it needs to start at zero): calls that overlap on one
 * GPU (different streams, or different host threads without ordering) race
 * on it and must be serialised by the caller.  Calls on different GPUs do
 * not interact.
 *
 * Errors: as ttsvd_tsqr_r, plus TTSVD_EINVAL when the shape needs more
 * than TTSVD_NOALLOC_SCRATCH_BYTES of tree storage
 * (ttsvd_tsqr_workspace_size(dtype, rows, cols) > the limit).
 */
#define TTSVD_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int ttsvd_tsqr_r_noalloc(const void *W, int dtype, int64_t rows, int64_t cols,
                         int64_t ld, double *R, int64_t ldr, hipStream_t stream);

/*
 * ttsvd_gemm_reshape -- fused tall-skinny matrix product and reshape.
 *
 * Defined in Sec. 4.1.2 (TSMM): Y <- reshape(W V, (rows/n_next, n_next*k)),
 * the step  W^(i-1) <- reshape(W^(i) V_{:,1:r}, ...)  of Algorithm 2.
 *
 *   W      device, rows x cols, column-major, ld >= rows, element type dtype.
 *   V      device, FP64, cols x k, column-major, leading dimension ldv >= cols.
 *   Y      device, element type dtype: the (rows/n_next) x (n_next*k) matrix
 *          reshape(W V) in column-major order with leading dimension
 *          ld_y >= rows/n_next.  Element (i, a) of W V is stored at
 *          Y[(i mod rows') + ld_y * (i div rows' + n_next * a)],
 *          rows' = rows / n_next.  Y must not overlap W or V.
 *   n_next must divide rows (n_next = 1 gives a plain product).
 *   FP64 data is accumulated in FP64; FP32 and BF16 data in FP32.
 *
 * Errors: TTSVD_EINVAL for non-positive sizes, rows % n_next != 0, short
 * leading dimensions or NULL pointers; TTSVD_EUNSUPPORTED for k > 256.
 */
int ttsvd_gemm_reshape(const void *W, int dtype, int64_t rows, int64_t cols,
                       int64_t ld, const double *V, int64_t ldv, int64_t k,
                       int64_t n_next, void *Y, int64_t ld_y,
                       hipStream_t stream);

/* Input tensor of ttsvd_decompose. */
typedef struct ttsvd_tensor {
    const void *data;    /* device, Fortran order, element type dtype       */
    int dtype;           /* ttsvd_dtype                                      */
    int64_t ld_last;     /* stride (in elements) of the last mode, >= n_1...n_{d-1};
                            0 means dense                                    */
    hipStream_t stream;  /* stream all work is enqueued on                   */
} ttsvd_tensor;

/*
 * Result of ttsvd_decompose.  Buffers are owned by the library and released
 * by ttsvd_tt_free.  Indices are 0-based: core j (j = 0..d-1) is the paper's
 * T^(j+1).
 */
typedef struct ttsvd_tt {
    int d;
    int64_t dims[TTSVD_MAX_D];
    int64_t ranks[TTSVD_MAX_D + 1];   /* ranks[0] = ranks[d] = 1              */
    double *cores[TTSVD_MAX_D];       /* device, FP64, (ranks[j], dims[j], ranks[j+1]), Fortran */
    double *sigma[TTSVD_MAX_D];       /* host: all singular values of the step that produced core j (j >= 1) */
    int64_t nsigma[TTSVD_MAX_D];      /* their count K = min(rows, cols) (0 for j = 0) */
    double discarded2[TTSVD_MAX_D];   /* sum of the discarded sigma^2 of that step */
    double delta;                     /* truncation threshold delta = tol/sqrt(d-1) ||Sigma||_F */
    double norm_sigma;                /* ||Sigma||_F of the first step (= ||X||_F) */
    double err_bound;                 /* sqrt(sum_j discarded2[j]) >= ||X - X~||_F */
    void *priv;                       /* library internal                     */
} ttsvd_tt;

/*
 * ttsvd_decompose -- TT decomposition of a dense tensor (Algorithm 2).
 *
 *   X      input tensor (read only).
 *   dims   n_1..n_d (host array of d values, each >= 1).
 *   d      number of modes, 1 <= d <= TTSVD_MAX_D.
 *   r_max  maximal TT rank (>= 1, the REQUIRE clause of Algorithms 1 and 2).
 *   tol    relative tolerance eps >= 0; delta = eps/sqrt(d-1) * ||Sigma||_F
 *          of the first step; the rank of each step is min(r_max, r_delta),
 *          r_delta = min{j : sigma_{j+1}^2 + sigma_{j+2}^2 + ... <= delta^2},
 *          clamped to [1, K].  tol = 0 means no tolerance: r = min(r_max, K).
 *   out    filled on success (see ttsvd_tt); release with ttsvd_tt_free.
 *
 * On return all work on X->stream has completed (the call synchronises it).
 * Errors: TTSVD_EINVAL (bad sizes, product of dims overflow, NULL pointers),
 * TTSVD_EUNSUPPORTED (dtype), TTSVD_ENOMEM, TTSVD_EHIP, TTSVD_ENONFINITE.
 */
int ttsvd_decompose(const ttsvd_tensor *X, const int64_t *dims, int d,
                    int64_t r_max, double tol, ttsvd_tt *out);

/*
 * ttsvd_decompose_two_sided -- the two-sided TSQR TT-SVD (Algorithm 4,
 * Sec. 3.1.3).  Steps alternate between the right-most and the left-most
 * remaining mode (i = d, 1, d-1, 2, ...); a left step takes the Q-less TSQR
 * of the transposed left unfolding, and the remainder is reordered by a
 * transpose between steps.  delta comes from the first step's ||Sigma||_F as
 * in Algorithm 2.  Same arguments and result as ttsvd_decompose, except that
 * sigma[j], nsigma[j] and discarded2[j] belong to the step that chose
 * ranks[j] (for j > the middle core these are the right steps, as in
 * ttsvd_decompose); cores left of the middle have orthonormal columns as
 * (r_{j-1} n_j) x r_j matrices, cores right of it orthonormal rows.  d <= 2
 * is Algorithm 2 itself.  Every step must have at most 1024 columns and keep
 * at most 256 (rank upper bounds); dense last mode only.  Synchronises
 * X->stream.  Errors as ttsvd_decompose (TTSVD_EUNSUPPORTED for the limits).
 */
int ttsvd_decompose_two_sided(const ttsvd_tensor *X, const int64_t *dims, int d,
                              int64_t r_max, double tol, ttsvd_tt *out);

/*
 * ttsvd_decompose_alg1 -- Algorithm 1 (the original TT-SVD, Sec. 3.1.1) on
 * the GPU, the in-house comparator that measures what the QR trick of
 * Algorithm 2 saves.  Every step takes the full SVD of the unfolding W^(i)
 * itself (rocSOLVER GESVD with its QR preprocessing off), the rank rule with
 * delta = eps/sqrt(d-1) ||X||_F (||X||_F^2 from the first step's singular
 * values), core T^(i) = reshape(V_r^T) and W^(i-1) = reshape(U_r Sigma_r).
 * Same arguments and result as ttsvd_decompose; FP64 input only, dense last
 * mode (ld_last 0 or equal to the leading extent), every unfolding within
 * 32-bit rocSOLVER sizes.  Synchronises X->stream.  Errors: TTSVD_EINVAL,
 * TTSVD_EUNSUPPORTED (dtype, padded stride, sizes), TTSVD_ENOMEM, TTSVD_EHIP
 * (also when GESVD does not converge), TTSVD_ENONFINITE.
 */
int ttsvd_decompose_alg1(const ttsvd_tensor *X, const int64_t *dims, int d,
                         int64_t r_max, double tol, ttsvd_tt *out);

/*
 * Caller-provided buffers for ttsvd_decompose (Algorithm 2, whose REQUIRE /
 * ENSURE clauses fix the inputs and outputs; the buffers are only where the
 * intermediate unfoldings W^(i) and the cores T^(i) live).
 *
 * ttsvd_workspace_size -- bytes of device workspace a decomposition of a
 * tensor with these dims, r_max and element type needs: the two ping-pong
 * work matrices W^(i) (sized for the rank upper bounds min(r_max, ...)), the
 * triangular factor R, the TSQR reduction tree, the SVD scratch, the singular
 * values and the per-step device state.  0 for invalid arguments.
 *
 * ttsvd_cores_size -- FP64 values the cores need at the rank upper bounds:
 * sum_j r_{j-1} n_j r_j with r_j = min(r_max, n_1...n_j, n_{j+1}...n_d, ...)
 * as the no-tolerance rule gives them.  0 for invalid arguments.
 */
size_t ttsvd_workspace_size(const int64_t *dims, int d, int64_t r_max, int dtype);
size_t ttsvd_cores_size(const int64_t *dims, int d, int64_t r_max);

/*
 * ttsvd_decompose_ws -- ttsvd_decompose (Algorithm 2) with caller-owned
 * device buffers, so the call makes no device allocation and no device free:
 *
 *   ws, ws_bytes       device workspace, 256-byte aligned, ws_bytes >=
 *                      ttsvd_workspace_size(dims, d, r_max, X->dtype).  Its
 *                      contents on entry do not matter; on return they are
 *                      undefined.  It must not overlap X or cores.
 *   cores, cores_doubles  device FP64 buffer of cores_doubles >=
 *                      ttsvd_cores_size(dims, d, r_max) values; out->cores[j]
 *                      point into it (core j at the offset of the rank upper
 *                      bounds of the cores left of it).  It stays owned by the
 *                      caller: ttsvd_tt_free releases only the host arrays of
 *                      out, and the cores stay valid until the caller reuses
 *                      or frees the buffer.
 *
 * Everything else (arguments, outputs, synchronisation of X->stream before
 * returning, errors) is as in ttsvd_decompose; additionally TTSVD_EINVAL for
 * NULL, short or misaligned buffers.  One pinned host staging buffer per
 * calling thread is allocated on the thread's first call and reused.  Two
 * calls that use the same ws at the same time race.
 */
int ttsvd_decompose_ws(const ttsvd_tensor *X, const int64_t *dims, int d, int64_t r_max,
                       double tol, void *ws, size_t ws_bytes, double *cores,
                       size_t cores_doubles, ttsvd_tt *out);

/*
 * Thick-bounds variant (Algorithm 3, Sec. 3.1.3 "Thick-bounds variant").
 *
 * ttsvd_thick_bounds_k -- number k of right-most modes to combine: the
 * smallest k in 1..d whose product m = n_{d-k+1} ... n_d satisfies
 * m >= max(m_min, r_est / f1_min), k = d if none does (the reading of the
 * threshold that reproduces Table 2).  dims: d host values; m_min >= 1;
 * 0 < f1_min <= 1; r_est >= 1 (an estimate of the first TT rank, e.g. r_max).
 * Writes k and m; errors: TTSVD_EINVAL (bad arguments, overflow of m).
 */
int ttsvd_thick_bounds_k(const int64_t *dims, int d, int64_t m_min, double f1_min,
                         int64_t r_est, int *k, int64_t *m);

/*
 * ttsvd_decompose_thick -- thick-bounds TT decomposition (Algorithm 3):
 * k, m from ttsvd_thick_bounds_k(dims, d, m_min, f1_min, r_max); Algorithm 2
 * (ttsvd_decompose, same r_max and tol) on X read as the tensor
 * (n_1, ..., n_{d-k}, m) -- the same memory in Fortran order -- and then on
 * its last core Tbar, read as the tensor (r_{d-k} n_{d-k+1}, n_{d-k+2}, ...,
 * n_d); the first core of the second decomposition is core d-k+1 of the
 * result.  k <= 1 or k >= d is ttsvd_decompose itself.
 *
 * out is a d-mode result as from ttsvd_decompose: sigma[j] and discarded2[j]
 * of the combined block's inner boundaries are those of the TT-SVD of Tbar;
 * delta and norm_sigma are the first decomposition's; err_bound =
 * e_1 + sigma_1 e_2 >= ||X - X~||_F, e_i = sqrt(sum of discarded sigma^2) of
 * each decomposition and sigma_1 the largest singular value at the block
 * boundary (X = L Tbar with ||L||_2 = sigma_1).  Without ranks cut inside the
 * block the result equals ttsvd_decompose's up to rounding.  All work runs on
 * X->stream, synchronised before returning; errors as ttsvd_decompose, plus
 * TTSVD_EINVAL for bad m_min / f1_min and TTSVD_EUNSUPPORTED for a padded
 * last-mode stride (X->ld_last other than 0 or n_1 ... n_{d-1}) when modes are
 * combined.  Release with ttsvd_tt_free.
 */
int ttsvd_decompose_thick(const ttsvd_tensor *X, const int64_t *dims, int d,
                          int64_t r_max, double tol, int64_t m_min, double f1_min,
                          ttsvd_tt *out);

/*
 * Batched form: Algorithm 2 applied independently to `count` tensors of
 * different shapes in one persistent cooperative launch.  All tensors advance
 * one TT step per round; the phases of a round (TSQR tree levels, small SVD
 * with truncation, TSMM + reshape) run the work units of every tensor over the
 * whole GPU, and each tensor's rank decision stays on the device.
 */
typedef struct ttsvd_batch_config {
    int grid;        /* workgroups of the persistent launch; 0 = all co-resident ones */
    int tile_set;    /* register tiling of the TSQR bodies: 0 (rows per lane 8 for
                        m <= 8; 16, 8, 4, 2 for the 16-, 32-, 64- and 128-column
                        buckets) for every dtype; 1 (half of those) for FP32 */
    int min_tiles;   /* a TSQR slice spans at least this many row tiles (>= 1)      */
    int max_slices;  /* TSQR slices per tensor and tree level at most (>= 1)        */
} ttsvd_batch_config;

/* The configuration used when no tuned one is known; returns TTSVD_OK. */
int ttsvd_batch_default_config(ttsvd_batch_config *cfg);

/*
 * ttsvd_decompose_batch -- TT decomposition of count tensors (Algorithm 2).
 *
 *   count  number of tensors, 1 <= count <= 4096.
 *   X      count input tensors (device, read only), all of the same dtype;
 *          X[t].stream is ignored.
 *   d      count mode counts (host), 1 <= d[t] <= TTSVD_MAX_D.
 *   dims   the dims of all tensors concatenated (host, sum of d[t] values).
 *   r_max  count maximal ranks (host, >= 1);  tol: count tolerances (host,
 *          >= 0), both as in ttsvd_decompose.
 *   cfg    tuning knobs, or NULL for the configuration ttsvd_batch_autotune
 *          found for this exact batch in this process (else the default).
 *   stream stream all work is enqueued on; synchronised before returning.
 *   out    count results, each released with ttsvd_tt_free (the cores of
 *          one call share a device allocation that the last free releases).
 *
 * Every step of every tensor must have at most 128 columns (n_j r_j <= 128
 * for the rank upper bounds min(r_max, ...)); larger problems belong to
 * ttsvd_decompose.  Errors: TTSVD_EINVAL, TTSVD_EUNSUPPORTED (mixed dtypes,
 * more than 128 columns), TTSVD_ENOMEM, TTSVD_EHIP, TTSVD_ENONFINITE (then
 * no result is returned).
 */
int ttsvd_decompose_batch(int count, const ttsvd_tensor *X, const int *d,
                          const int64_t *dims, const int64_t *r_max,
                          const double *tol, const ttsvd_batch_config *cfg,
                          hipStream_t stream, ttsvd_tt *out);

/*
 * ttsvd_batch_autotune -- time the batch under each candidate configuration
 * (TSQR slice sizes and counts, tile sets built for the dtype), return the
 * fastest in *best and its time in *best_ms (may be NULL): the host wall
 * time of one call plus the release of its results, the span a caller sees.
 * The choice is remembered for later
 * ttsvd_decompose_batch calls with cfg = NULL on the same batch (same count,
 * dtype, dims, r_max, tol and strides).  The decompositions it runs are
 * discarded.  Errors as ttsvd_decompose_batch.
 */
int ttsvd_batch_autotune(int count, const ttsvd_tensor *X, const int *d,
                         const int64_t *dims, const int64_t *r_max,
                         const double *tol, hipStream_t stream,
                         ttsvd_batch_config *best, double *best_ms);

/*
 * Serving runtime: requests that arrive over time are admitted while the sum
 * of their device footprints (ttsvd_footprint_bytes) stays within a budget
 * and run by worker threads, each on its own stream.  Continuous batching:
 * small requests (every step at most 128 columns, at most batch_max_elems
 * elements, dense) wait in their own FIFO, and whenever no batched launch is
 * running a free worker decomposes all of them that fit (up to max_batch) in
 * one batched launch, so requests arriving meanwhile join the next one.  The
 * other requests wait in FIFO order and run alone on the other workers.
 * Timestamps are seconds of ttsvd_server_clock().
 */
typedef struct ttsvd_server ttsvd_server;

typedef struct ttsvd_server_config {
    size_t hbm_budget;        /* bytes of workspace + outputs admitted at once (> 0)  */
    int workers;              /* worker threads / streams, 1..64                      */
    int max_batch;            /* requests per batched launch (1: never batch)         */
    int64_t batch_max_elems;  /* largest tensor eligible for a batched launch         */
} ttsvd_server_config;

typedef struct ttsvd_completion {
    uint64_t ticket;          /* from ttsvd_server_submit                            */
    int status;               /* TTSVD_OK or the error of the decomposition          */
    int batch_size;           /* requests in the launch that ran it                  */
    int batched;              /* 1: ran in a batched launch, 0: ttsvd_decompose      */
    double t_submit, t_start, t_done;
    char message[160];        /* the error message when status != TTSVD_OK          */
    ttsvd_tt tt;              /* result (status TTSVD_OK); release with ttsvd_tt_free */
} ttsvd_completion;

/* Defaults: 64 GiB budget, 4 workers, batches of up to 512, 2^24 elements. */
int ttsvd_server_default_config(ttsvd_server_config *cfg);
/* Start a server on the calling thread's current device.  Errors: TTSVD_EINVAL. */
int ttsvd_server_create(const ttsvd_server_config *cfg, ttsvd_server **out);
/* Queue a decomposition of X (device memory that must stay valid and unchanged
 * until its completion is returned).  X->stream is the stream that produced
 * X (a stream of the server's device, NULL = the legacy default stream): the
 * call records an event on it, and the request's work starts only after
 * everything enqueued there before the call, so the producer need not
 * synchronise before submitting.  The request itself runs on a worker's
 * stream.  Arguments as in ttsvd_decompose; *ticket identifies the request.
 * Errors: TTSVD_EINVAL, TTSVD_EUNSUPPORTED, TTSVD_EHIP (the event could not
 * be recorded on X->stream). */
int ttsvd_server_submit(ttsvd_server *s, const ttsvd_tensor *X, const int64_t *dims, int d,
                        int64_t r_max, double tol, uint64_t *ticket);
/* Move up to max finished requests into out (waiting up to wait_ms for the
 * first one); *n receives the count. */
int ttsvd_server_poll(ttsvd_server *s, ttsvd_completion *out, int max, int wait_ms, int *n);
/* Requests submitted and not yet finished. */
int64_t ttsvd_server_pending(ttsvd_server *s);
/* Finish every queued request, stop the workers and free unpolled results. */
void ttsvd_server_destroy(ttsvd_server *s);
/* The steady clock of the completion timestamps, in seconds. */
double ttsvd_server_clock(void);

/* Release the buffers of a ttsvd_tt filled by ttsvd_decompose or
 * ttsvd_decompose_batch (NULL-safe).  Library-owned cores go back to the
 * library's device buffer cache after the device is synchronised (as hipFree
 * would); they are not returned to the driver, so repeated calls reuse them. */
void ttsvd_tt_free(ttsvd_tt *tt);

/* Device bytes ttsvd_decompose allocates for this problem (work matrices,
 * triangular factors, SVD scratch and the output cores), excluding X. */
size_t ttsvd_footprint_bytes(const int64_t *dims, int d, int64_t r_max,
                             int dtype);

/* Static description of a status code. */
const char *ttsvd_strerror(int code);

/* Message of the last error on the calling thread ("" if none). */
const char *ttsvd_last_error(void);

/* Library version string. */
const char *ttsvd_version(void);

/*
 * Kernel timing.  Not part of the method: measurement support for the
 * roofline report of Sec. 4 (achieved bytes and flops per kernel against the
 * hardware limits).  While enabled, every kernel the library launches is
 * bracketed by HIP events recorded on its launch stream, together with the
 * algorithmic bytes and flops of that launch (a TSQR level reads its input
 * once; the TSMM reads W once and writes Y once; flops 2 n m^2 and 2 n m k).
 */
typedef struct ttsvd_kernel_stat {
    char name[96];        /* kernel instance, e.g. "tsqr_rows<64,1,f64>"     */
    int64_t launches;
    double total_ms;      /* sum of event-measured launch durations          */
    double bytes;         /* sum of algorithmic bytes                        */
    double flops;         /* sum of algorithmic flops                        */
} ttsvd_kernel_stat;

/* Turn recording on (on != 0) or off; returns TTSVD_OK. */
int ttsvd_profile_enable(int on);
/* Drop all records. */
void ttsvd_profile_reset(void);
/* Aggregate the records by kernel name (waits for their events).  Writes up
 * to max_stats entries to stats and the number of distinct kernels to
 * *n_stats.  Errors: TTSVD_EINVAL (NULL pointers), TTSVD_EHIP. */
int ttsvd_profile_read(ttsvd_kernel_stat *stats, int max_stats, int *n_stats);

/*
 * Machine micro-benchmarks: the measured denominators of the roofline report
 * (the analog of the machine characterisation of Sec. 5, Table 1: load,
 * store, copy and triad memory bandwidth and the FP64 FMA rate).  Not part of
 * the method.
 *
 *   kind   TTSVD_MB_LOAD (sum of a[i]), TTSVD_MB_STORE (a[i] = 0),
 *          TTSVD_MB_COPY (b[i] = a[i]), TTSVD_MB_TRIAD (a[i] = b[i] + s c[i]),
 *          TTSVD_MB_FMA (independent FP64 FMA chains, no memory traffic).
 *   buf    device buffer of `bytes` bytes, split into 1, 2 or 3 equal arrays
 *          (load/store, copy, triad); zero-filled by the caller for LOAD.
 *          For FMA it must hold one double (never written in practice).
 *   reps   timed launches after one untimed warm-up, on `stream`.
 *   out    host: out[0] = milliseconds per launch (HIP events),
 *          out[1] = bytes moved (or flops for FMA) per launch.
 * Synchronises the stream.  Errors: TTSVD_EINVAL, TTSVD_EHIP.
 */
enum {
    TTSVD_MB_LOAD = 0,
    TTSVD_MB_STORE = 1,
    TTSVD_MB_COPY = 2,
    TTSVD_MB_TRIAD = 3,
    TTSVD_MB_FMA = 4
};
int ttsvd_machine_bench(int kind, void *buf, size_t bytes, int reps, hipStream_t stream,
                        double *out);

#ifdef __cplusplus
}
#endif

#endif /* TTSVD_H */
