/*
 * swalign.h -- C ABI of the MI355X (gfx950) library for rigid alignment of
 * images in sliced 2-Wasserstein distance.
 *
 * The method (Shi, Singer, Verbeke, "Fast rigid alignment of heterogeneous
 * images in sliced Wasserstein distance"):
 *   1. project every image onto n angles                        (Sec. 2.2-2.3)
 *   2. turn every projection into a CDF and a table of Q quantiles  (Sec. 2.3)
 *   3. cross-correlate two quantile tables along the angle axis by FFT, one
 *      correlation per quantile row summed over rows               (Sec. 2.3,
 *      fast computation over rotations)
 *   4. correct each rotation lag with the least-squares translation, which
 *      follows from the translation equivariance of SW2           (Thm 3.2)
 *   5. take the argmin over the rotation grid.
 * The problem solved for a reference f and a target g is
 *   argmin over (s, theta) of d(f, T_s R_theta g)              (Sec. 1.1)
 * with theta restricted to the grid 2 pi l / n.
 *
 * Conventions used throughout:
 *   - images are row-major L x L float32; pixel (i, j) sits at
 *     x = (j - (L-1)/2) h, y = (i - (L-1)/2) h, h = 2/L (x along +column,
 *     y along +row); only pixels with x^2 + y^2 <= (1-h)^2 are used and
 *     negative values count as 0;
 *   - angle k is theta_k = 2 pi k / n; detector bin b has centre
 *     -1 + (b + 1/2) h; quantile level j is (j + 1/2)/Q (or j/Q);
 *   - a result (rot_index = l, shift_px = s) means f ~ T_s R_theta g with
 *     theta = 2 pi l / n; sw2sq is the squared distance (1/(nQ)) times the
 *     squared Frobenius norm of the table difference (Sec. 2.3).
 *
 * Memory: every array argument is a DEVICE pointer unless marked "host".  The
 * caller owns all arrays it passes; the library never frees them.  The
 * library owns its scratch (angle spectra, tables), released by
 * sw_ctx_destroy.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 * Compute calls are asynchronous on that stream.  One context's scratch is
 * shared by its calls: calls on one context must be issued on one stream (or
 * otherwise ordered); use one context per concurrent stream.
 *
 * Errors: every call returns sw_status; no C++ exception crosses the ABI.
 * sw_last_error() returns a thread-local message for the last failure.
 * Whole-call errors (bad geometry, null pointers, device failures) fail the
 * call; per-image problems (zero mass after clipping and masking, a
 * non-finite pixel) are reported in sw_result.status and the call succeeds.
 */
#ifndef SWALIGN_H
#define SWALIGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SW_OK = 0,
    SW_NOT_READY = 1,      /* serving: result not finished yet */
    SW_E_INVALID = -1,     /* bad argument or geometry */
    SW_E_NOMEM = -2,       /* allocation failed, or a request exceeds the budget */
    SW_E_DEVICE = -3,      /* HIP runtime error */
    SW_E_UNSUPPORTED = -4, /* valid but not implemented combination */
    SW_E_BUSY = -5         /* serving queue full (back-pressure) */
} sw_status;

/* Quantile levels z_j: midpoint (j + 1/2)/Q (default) or left j/Q, the
   left Riemann sum of the paper's error analysis (App. A, E3). */
typedef enum { SW_LEVELS_MIDPOINT = 0, SW_LEVELS_LEFT = 1 } sw_levels;

/* Rotation + closed-form translation (default), or rotation only, which is
   the paper's own objective (Sec. 2.3, discrete SW2 over rotations), or the
   max-sliced objective, rotation only (extended alignment results: the
   largest per-angle W2^2 instead of the mean, M(l) = max_k (1/Q) sum_j
   (U[j][k] - V[j][(k+l) mod n])^2; the shift is reported as 0).  The
   max-sliced mode takes n_angles a multiple of 16 up to 128 (16, 32, 48,
   64, 96, 128); its top_k lags (from an FP32
   matrix-core estimate of every lag) are rescored as direct residuals, and
   the curve holds the estimate. */
typedef enum { SW_MODE_ROT_TRANS = 0, SW_MODE_ROT_ONLY = 1, SW_MODE_MAX_SLICED = 2 } sw_mode;

/* FP32 everywhere, or FP32 tables with a BF16 correlation (FP32 accumulate)
   and an FP32 rescore of the top_k lags. */
typedef enum { SW_PREC_FP32 = 0, SW_PREC_BF16_SPLIT = 1 } sw_precision;

/* Projection filter of the alignment: none (SW2) or the ramp filter |xi|
   of Sec. 2.2 (ramp-filtered SW2 of Sec. 2.3: each filtered slice split into
   its positive and negative parts, each normalised and compared on its own,
   the two distances summed). */
typedef enum { SW_FILTER_NONE = 0, SW_FILTER_RAMP = 1 } sw_filter;

/* Per-result status: zero mass after clipping and masking, a non-finite
   input value, or a pair index outside the table sets. */
enum { SW_RESULT_OK = 0, SW_RESULT_ZERO_MASS = 1, SW_RESULT_NONFINITE = 2, SW_RESULT_BAD_PAIR = 3 };

/* Geometry.  Valid: 8 <= L <= 256; n_angles a multiple of 8, at most 512,
   whose only prime factors are 2 and 3; n_quantiles a multiple of 4 in
   [8, 512]. */
typedef struct {
    int32_t L;
    int32_t n_angles;
    int32_t n_quantiles;
    int32_t levels; /* sw_levels */
} sw_geom;

/* One alignment result (24 bytes). */
typedef struct {
    int32_t rot_index;  /* l* in [0, n) */
    float theta_rad;    /* 2 pi l* / n */
    float shift_px[2];  /* s* in pixels: [0] along +column (x), [1] along +row (y) */
    float sw2sq;        /* squared SW2 at (l*, s*), unit-disk coordinates */
    int32_t status;     /* SW_RESULT_* */
} sw_result;

/* Context: binds a device and owns scratch.  tune_json (host, nullable) is a
   path to a JSON file with optional keys: "tiles" (the table written by
   sw_autotune), "small_batch": calls on fewer images than this take the
   split launches (several blocks per image; default: the number of compute
   units), "tables_images_per_block": 1 or 2 (default 2), the images one
   block of the fused sw_tables / sw_tables_rf kernels projects from the same
   strips where the geometry allows two, and "align_kernel": "generic", which
   keeps sw_align_batch on the LDS-FFT pair kernel for n_angles = 128 instead
   of the register-FFT one (the two agree to FP32 rounding), or "block128",
   which runs the register-FFT alignment with one pair per block instead of
   one pair per wave (same arithmetic, sums in another order).  The first
   three change launch shapes only, never results. */
/* Scratch: the context owns one scratch buffer (grown on demand) that the
   calls needing it share: sw_tables / sw_tables_rf when they take their
   chunked or small-batch path, sw_align_batch (except the max-sliced mode)
   and sw_align_stacks, sw_project_fourier(_at) and sw_tables_fourier(_at);
   sw_project, sw_ramp, sw_quantiles and sw_quantiles_rf never.  Calls on
   different streams may overlap only when at most one of them uses scratch (e.g. the tables of a single
   reference on a side stream next to the fused tables of a large image
   batch); otherwise order them with events. */
sw_status sw_ctx_create(void **ctx, int device, const char *tune_json);
sw_status sw_ctx_destroy(void *ctx);
const char *sw_last_error(void);
const char *sw_version(void);

/* The work plan of the line projection (Sec. 2.2/2.3, step 1) for side L and
   n angles, as every projection launch of (L, n) uses it: host memory only,
   no context and no device work (for inspection and tests).  Items are
   (slot angle m <= n/8, bin b) pairs, item = m L + b; a task is 64 lanes,
   eight units of 8 consecutive bins of one slot.  perm[t 64 + l] = the item
   of lane l of task t, or -1; [row_lo[t], row_hi[t]] = the image rows task t
   reads (every row where one of its items' lines has a pixel of non-zero
   weight inside the disk; row_lo > row_hi for a task with none).  *ntasks is
   set first; the arrays (cap_tasks tasks; NULL with cap_tasks = 0 to query
   the count) are filled when cap_tasks >= *ntasks, else SW_E_INVALID.  The
   plan does not change results: rows outside a task's range add only zeros. */
sw_status sw_projection_plan(int32_t L, int32_t n, int32_t cap_tasks, int32_t *perm /*host*/,
                             int32_t *row_lo /*host*/, int32_t *row_hi /*host*/,
                             int32_t *ntasks /*host*/);

/* Step 1, line projection (Sec. 2.2 Radon transform, Sec. 2.3 columns of U).
   pmf[g][k][b] = sum over masked pixels of max(F,0) * max(0, 1 - |p.d_k - c_b|/h)
   with d_k = (cos theta_k, -sin theta_k) and c_b the centre of bin b: each
   pixel deposits its value into the two bins around its projected position
   by linear interpolation.  Unnormalised (column sums equal the image mass).
   img: [N][L][L] float32, pmf: [N][n][L] float32 (caller-allocated).
   An image holding a non-finite value yields an all-NaN projection. */
sw_status sw_project(void *ctx, const float *img, int64_t N, const sw_geom *g /*host*/,
                     float *pmf, void *stream);

/* Step 2, CDF and quantile table (Sec. 2.3: cumulative sums, then ICDF by
   linear interpolation; generalised inverse inf{t : F(t) >= z}, App. A).
   Per column k: C[b] = (sum_{b'<=b} pmf[k][b'])/m_k accumulated in FP64,
   b* = min{b : C[b] >= z_j}, qt[j][k] = t_{b*} + h (z_j - C[b*-1]) /
   (C[b*] - C[b*-1]) clamped to the bin, t_b = -1 + b h.
   pmf: [N][n][L] float32, qt: [N][Q][n] float32.
   aux (nullable): [N][4] float64 = { mass (NaN if non-finite), E = sum qt^2,
   Re a, Im a } with a = (1/n) sum_k qbar_k (cos theta_k, -sin theta_k),
   qbar_k the mean of column k (the translation moment). */
sw_status sw_quantiles(void *ctx, const float *pmf, int64_t N, const sw_geom *g /*host*/,
                       float *qt, double *aux, void *stream);

/* Steps 1 and 2 fused: images straight to quantile tables, the projection
   never leaving the chip.  Same outputs as sw_project followed by
   sw_quantiles. */
sw_status sw_tables(void *ctx, const float *img, int64_t N, const sw_geom *g /*host*/, float *qt,
                    double *aux, void *stream);

/* Ramp filter of projections (Sec. 2.2, optional high-pass step; the
   ramp-filtered distance of Sec. 2.3).  The filter |xi| is sampled on the
   2L-point frequency grid of the detector with the DC term zero and applied
   to each column zero-padded to 2L, i.e. the cyclic convolution
     out[g][k][b] = sum_{b'} h[(b - b') mod 2L] pmf[g][k][b'],
     h[0] = L/2, h[m] = -1/(2L sin^2(pi m / 2L)) for odd m, 0 for even m != 0,
   kept on the L detector bins; any positive scale of the filter cancels in
   the normalised parts.  Computed in FP32 on the matrix cores.
   pmf, out: [N][n][L] float32 (out may equal pmf).  NaN columns stay NaN. */
sw_status sw_ramp(void *ctx, const float *pmf, int64_t N, const sw_geom *g /*host*/, float *out,
                  void *stream);

/* Step 2 for ramp-filtered projections: each column of pf is split into its
   positive part max(pf, 0) and its absolute negative part max(-pf, 0), each
   part is inverted as in sw_quantiles (normalised on its own), and the two
   tables are stacked: qt[g][j][k] for j < Q is the positive part, j >= Q the
   negative part.  2 * n_quantiles must not exceed 512.
   pf: [N][n][L] float32, qt: [N][2Q][n] float32.
   aux (nullable): [N][4] float64 = { the smallest part mass over all columns
   (0 when a part is empty somewhere: such an image aligns with status
   SW_RESULT_ZERO_MASS; NaN if a value is NaN), E and Re a, Im a of the
   stacked table }. */
sw_status sw_quantiles_rf(void *ctx, const float *pf, int64_t N, const sw_geom *g /*host*/,
                          float *qt, double *aux, void *stream);

/* Images to stacked ramp-filtered tables: sw_project, sw_ramp and
   sw_quantiles_rf in one call (through a bounded scratch buffer). */
sw_status sw_tables_rf(void *ctx, const float *img, int64_t N, const sw_geom *g /*host*/,
                       float *qt, double *aux, void *stream);

/* Step 1 by the Fourier slice theorem (Sec. 2.2; the projections of
   Sec. 2.3 through a NUFFT and a 1-D inverse DFT), discretised as in the
   appendix's fixed-angle error theorem with NUFFT precision.  With the same
   pixel masses m as sw_project (positive part inside the disk), pixel
   centres x_ij, h = 2/L, L = 2M, d_k = (cos theta_k, -sin theta_k):
     yhat_k(j) = S_j(d_k) sum_pixels m exp(-i j pi d_k . x),  j = -M .. M-1,
   with S_j the transform of one pixel cell, sinc(j pi d_x h/2)
   sinc(j pi d_y h/2); pmf[g][k][b] = max(0, h Re g_k(c_b)) for the
   trigonometric polynomial g_k(s) = (1/2) sum_j yhat_k(j) exp(i j pi s) at
   the bin centres c_b (negative lobes clipped; column sums equal the image
   mass up to the clipped lobes).  The slices are evaluated by a type-2
   NUFFT (grid oversampled by 2, exponential-of-semicircle kernel of width
   7: relative error about 1e-6 before FP32 rounding), two slices per FP32
   inverse FFT.  L must be even with prime factors 2 and 3 only (8, 12, 16,
   18, 24, ..., 96, ..., 192, 256; mixed-radix transforms of lengths L and
   2L).  Uses the context scratch.
   img: [N][L][L] float32, pmf: [N][n][L] float32.  An image holding a
   non-finite value yields an all-NaN projection. */
sw_status sw_project_fourier(void *ctx, const float *img, int64_t N, const sw_geom *g /*host*/,
                             float *pmf, void *stream);

/* sw_project_fourier followed by sw_quantiles, through a bounded scratch
   buffer: images to quantile tables with the Fourier-slice projector. */
sw_status sw_tables_fourier(void *ctx, const float *img, int64_t N, const sw_geom *g /*host*/,
                            float *qt, double *aux, void *stream);

/* The same projections at n_angles explicit directions theta[k] (radians,
   any values; d_k = (cos theta_k, -sin theta_k)) instead of 2 pi k / n, each
   slice computed on its own.  This is the Monte-Carlo SW of the extended
   alignment results: draw the directions uniformly on the circle, sort
   them, build both images' tables with the same theta, and run
   sw_align_batch in SW_MODE_ROT_ONLY (the column-shift scan unchanged, lag
   l read as the rotation 2 pi l / n; the closed-form translation assumes
   equispaced directions).  sw_tables_fourier_at computes the quantile
   tables with aux moments over these directions.  theta: host
   [n_angles] float64, read during the call (the slice tables are cached
   per distinct theta in the context).  Otherwise as sw_project_fourier and
   sw_tables_fourier. */
sw_status sw_project_fourier_at(void *ctx, const float *img, int64_t N, const sw_geom *g /*host*/,
                                const double *theta /*host*/, float *pmf, void *stream);
sw_status sw_tables_fourier_at(void *ctx, const float *img, int64_t N, const sw_geom *g /*host*/,
                               const double *theta /*host*/, float *qt, double *aux,
                               void *stream);

/* Steps 3-5: alignment of table pairs.
   For each pair (r, g): the angle spectra of both tables, the correlation
   C(l) = sum_{j,k} U[j][k] V[j][(k+l) mod n] for all l by FFT along the angle
   axis, D0(l) = (E_U + E_V - 2 C(l))/(nQ), b(l) = a_U - e^{i theta_l} a_V,
   s*(l) = 2 b(l), D*(l) = D0(l) - 2|b(l)|^2 (ROT_TRANS) or D0(l)
   (ROT_ONLY), l* = argmin D*(l) (ties to the smallest l), then sw2sq
   recomputed at (l*, s*) as a direct FP32 residual sum.  With top_k > 1
   the top_k lags are rescored and the smallest rescored value wins.
   pairs: [n_pairs][2] int64 (ref index, img index) or NULL for all
   ref x img in row-major order (pair p = r * n_img + g).
   out: [P] sw_result; curve (nullable): [P][n] float32, D*(l). */
typedef struct {
    const float *ref_qt;   /* [n_ref][Q][n] */
    const double *ref_aux; /* [n_ref][4] */
    int64_t n_ref;
    const float *img_qt;   /* [n_img][Q][n] */
    const double *img_aux; /* [n_img][4] */
    int64_t n_img;
    const int64_t *pairs;  /* [n_pairs][2] or NULL */
    int64_t n_pairs;
    sw_geom geom;
    int32_t mode;          /* sw_mode */
    int32_t prec;          /* sw_precision */
    int32_t top_k;         /* 1..8; 0 means 1 for FP32 and 4 for BF16_SPLIT */
    int32_t filter;        /* sw_filter; SW_FILTER_RAMP: the tables are the stacked
                              [2Q][n] tables of sw_tables_rf (geom.n_quantiles = Q,
                              2Q <= 512), and sw2sq and the curve are the
                              ramp-filtered distance: the sum over both parts of
                              (1/(nQ)) sum_{j,k} (U - V - s.d_k)^2.  The rotation
                              and the shift minimise that sum; s* = 2 b(l) with
                              b from the column means of the stacked tables. */
} sw_batch;

sw_status sw_align_batch(void *ctx, const sw_batch *b /*host*/, sw_result *out, float *curve,
                         void *stream);

/* sw_align_batch for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   same arguments, same kernels, same results, but no allocation of any
   kind.  Its angle tables and scratch live in one fixed array per GPU
   (64 MiB of work area plus the angle tables of every admissible n_angles,
   held from the first sw_ctx_create on that GPU until the process ends).
   A call whose scratch need exceeds 64 MiB fails with SW_E_NOMEM before any
   launch: the 1-vs-many and pair-list forms need 8 (n/2+1) Q bytes per
   reference (plus 520 Q bytes per reference at n = 128: 133 KiB in all at
   n = Q = 128), the all-pairs BF16 form 4 (n/2+1) Q bytes per table of
   both sets plus 2 top_k bytes per pair (about 47 MiB for 2,000 x 2,000
   tables at n = Q = 64).  All calls on
   one GPU share the array: calls that overlap on one GPU (other streams,
   other contexts, other threads) race and must be ordered by the caller.
   Nothing in it needs clearing between calls. */
sw_status sw_align_batch_noalloc(void *ctx, const sw_batch *b /*host*/, sw_result *out,
                                 float *curve, void *stream);

/* Uneven batch: stacks of images of different geometry, each aligned
   against its own reference image (steps 1-5 for every image of every
   stack).  All stacks go through persistent mixed-geometry launches (one
   launch per stage for up to 64 stacks) whose blocks take work items from a
   device counter, largest L first; the projection strip tile per L comes from
   the autotuner's table when the context was created with one.
   Outputs are caller-allocated device arrays; results go to out[N] of each
   stack, with the reference and image tables left in ref_qt/ref_aux and
   qt/aux.  prec SW_PREC_BF16_SPLIT rounds the spectra to bfloat16 before
   the correlation and rescoring the top_k lags in FP32. */
typedef struct {
    const float *ref_img; /* [L][L] */
    const float *imgs;    /* [N][L][L] */
    int64_t N;
    sw_geom geom;
    float *ref_qt;        /* [Q][n] */
    double *ref_aux;      /* [4] */
    float *qt;            /* [N][Q][n] */
    double *aux;          /* [N][4] */
    sw_result *out;       /* [N] */
} sw_stack;

sw_status sw_align_stacks(void *ctx, const sw_stack *stacks /*host*/, int32_t n_stacks,
                          int32_t mode, int32_t prec, int32_t top_k, void *stream);

/* Autotuner: for each side L in Ls (geometry n = Q = L), times the mixed
   pipeline on n_images synthetic images and picks, one after the other, the
   projection strip height, the tables kernel's tasks per wave (5 or 6: the
   number of task groups an image is restaged for) and the blocks per
   compute unit of the per-pair alignment kernel (2, 4, 6 or 8), each the
   fastest given the ones before.  None of them changes a result.  The table
   is kept in the context and, when out_json is given, written there as
   {"tiles": {"L": {"R": rows, "tpw": tasks, "align_bpc": blocks, "ms": t}}}
   (tpw and align_bpc only when they differ from the defaults); pass that
   file to sw_ctx_create to reuse it.  A mixed launch of several L takes the
   tasks per wave and alignment blocks of its L with the most projection
   work.  Synchronises the device. */
sw_status sw_autotune(void *ctx, const int32_t *Ls /*host*/, int32_t nL, int64_t n_images,
                      const char *out_json /*host, nullable*/);

/* Serving: continuous batching of alignment requests (1 reference image +
   N images each, host memory).  A scheduler thread owned by the context
   admits queued requests in arrival order while the request fits in the HBM
   budget and a slot is free, copies its images to the device on a copy
   stream, and launches the admitted requests of one geometry together (at
   most max_per_step per step) through the mixed persistent kernels,
   replayed from a captured graph; with fewer per step than slots, the next
   step's copies run while the current step computes; requests that arrive
   while others run are admitted as slots and memory free up, so their work
   shares launches and overlaps on the device.  Reference tables with a
   non-zero ref_key stay cached in HBM (evicted least recently used when
   memory is needed).  Results are computed with the same kernels as
   sw_align_stacks, so a request's results do not depend on what else was in
   the batch.
   Contract: the caller keeps ref_img and imgs valid until sw_serve_poll
   returns SW_OK for the ticket or sw_serve_cancel returns.
   Errors: sw_serve_submit returns SW_E_NOMEM when the request alone exceeds
   the budget, SW_E_BUSY when max_queue requests are already waiting;
   sw_serve_poll returns SW_NOT_READY until the results are in `out`,
   SW_E_INVALID for an unknown or cancelled ticket, SW_E_DEVICE if the device
   work failed.  Calls are thread-safe. */
typedef struct {
    size_t hbm_budget_bytes; /* arena for images, tables, results and the cache */
    int32_t max_slots;       /* requests admitted at once (<= 64 per launch) */
    int32_t prec;            /* sw_precision */
    int32_t top_k;           /* 0 = 1 for FP32, 4 for BF16_SPLIT */
    int32_t mode;            /* sw_mode */
    int32_t max_queue;       /* waiting requests before SW_E_BUSY */
    int32_t use_graphs;      /* 1: replay captured graphs, 0: plain launches */
    int32_t max_per_step;    /* requests per launch sequence (0: max_slots, at most 64);
                                below max_slots, the copies of the next step's requests
                                overlap the current step's kernels */
} sw_serve_cfg;

typedef struct {
    const float *ref_img; /* host [L][L] */
    const float *imgs;    /* host [N][L][L] */
    int64_t N;
    sw_geom geom;
    uint64_t ref_key;     /* 0 = reference tables not cached */
} sw_request;

/* Counters since sw_serve_start.  waited_memory / waited_slot: admitted
   requests that, at the head of the queue, had to wait because the arena
   had no room for them / because max_slots requests were in flight (a
   request may count in both). */
typedef struct {
    uint64_t submitted, admitted, completed, cancelled, failed;
    uint64_t steps, graph_launches, cache_hits, evictions;
    int64_t pending, in_flight;
    size_t arena_used, arena_peak, arena_size;
    uint64_t waited_memory, waited_slot;
} sw_serve_stats;

sw_status sw_serve_start(void *ctx, const sw_serve_cfg *cfg /*host*/);
sw_status sw_serve_submit(void *ctx, const sw_request *r /*host*/, uint64_t *ticket /*host*/);
sw_status sw_serve_poll(void *ctx, uint64_t ticket, sw_result *out /*host [N]*/);
sw_status sw_serve_cancel(void *ctx, uint64_t ticket);
sw_status sw_serve_stats_get(void *ctx, sw_serve_stats *out /*host*/);
sw_status sw_serve_stop(void *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SWALIGN_H */
