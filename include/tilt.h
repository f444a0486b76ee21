/*
 * tilt.h -- C interface of the MI355X TILT solver (LADMAP with warm starts).
 *
 * Problem (Ren & Lin, arXiv 1205.5351, Eq. TILT_2 and Alg. 1): given a
 * grey-level image D and an initial transform tau0 of an m x n window, find
 * the transform tau, a low-rank texture A and sparse errors E with
 *
 *     min ||A||_* + lambda ||E||_1   s.t.   D o tau = A + E,
 *
 * by the outer loop of Alg. 1 (normalise, Jacobian, inner solve, Delta tau
 * from Eq. Delta_tau, tau += Delta tau) around the LADMAP inner loop of
 * Sec. 3.2 in the form of Sec. 4.2 (two J_perp products per iteration,
 * Y kept in span(J_perp)) with the variable warm start of Eq. warm_start and
 * Eq. warm_start_Y.  The extra constraints Q Delta tau = 0 of Sec. 4.3 fix
 * the image of the window centre and the area of the image of the window
 * to first order.
 *
 * Conventions shared by every entry point
 *   - image: row-major float32, pixel centres at integer (x = column,
 *     y = row); row_stride counts elements.  Height and width >= 2.
 *   - rectified grid: rows i = 0..m-1, columns j = 0..n-1 with centred
 *     coordinates u = j - (n-1)/2, v = i - (m-1)/2.
 *   - a transform is a 3x3 row-major homography H with
 *     (x, y, 1) ~ H (u, v, 1); H[2][2] = 1.  The affine model requires the
 *     last row (0, 0, 1).  Inside the solver tau lives in coordinates scaled
 *     by s = max(m, n)/2 about the image of the window centre; tau0 and the
 *     returned tau are always pixel homographies.
 *   - bilinear sampling; outside the image samples are clamped to the
 *     border and the gradient along the clamped axis is zero.
 *   - A and E are m x n row-major float32.
 *
 * Status codes: 0 = OK, > 0 = warning, < 0 = error.  No entry point throws
 * or aborts; each returns the worst per-patch status it saw.
 */
#ifndef TILT_H
#define TILT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum tilt_status {
    TILT_OK = 0,
    TILT_WARN_MAXITER = 1,     /* an inner loop stopped at max_inner       */
    TILT_PENDING = 2,          /* tilt_poll: request not finished yet      */
    TILT_ERR_ARG = -1,         /* invalid argument                         */
    TILT_ERR_NOMEM = -2,       /* device allocation failed / over budget   */
    TILT_ERR_DEVICE = -3,      /* HIP runtime error                        */
    TILT_ERR_SINGULAR = -4,    /* J^T J not positive definite (flat image) */
    TILT_ERR_NONFINITE = -5,   /* NaN/Inf in the iteration                 */
    TILT_ERR_TOO_LARGE = -6,   /* patch does not fit the on-chip SVT       */
    TILT_ERR_NOT_FOUND = -7    /* unknown ticket                           */
};

enum tilt_model { TILT_AFFINE = 6, TILT_PROJECTIVE = 8 };

/* Solver parameters.  Names follow the paper: lambda (Eq. TILT_2), eps1 and
 * eps2 (Eqs. Cond1, Cond2, rho), rho0 and mu_max (Eqs. mu, rho).  The paper
 * gives no values; defaults come from tilt_default_params(). */
typedef struct {
    double lambda;      /* <= 0: 1/sqrt(max(m, n))                            */
    double eps1;        /* Cond1 threshold, default 1e-5                      */
    double eps2;        /* Cond2 and rho threshold, default 1e-3              */
    double eps_outer;   /* outer stop when ||Delta tau||_2 < eps_outer
                           (scaled coordinates), default 1e-5                 */
    double mu0;         /* <= 0: 1.25 / ||D o tau||_2 at each inner start      */
    double rho0;        /* >= 1, default 1.5                                  */
    double mu_max;      /* default 1e10                                       */
    int max_inner;      /* default 2000                                       */
    int max_outer;      /* default 50                                         */
    int fixed_iters;    /* 1: run exactly max_outer x max_inner iterations
                           (stop tests evaluated but ignored)                 */
    int svt_mode;       /* 0: cold one-sided Jacobi SVT every iteration.
                           1: warm start: each SVT starts from the previous
                           SVT's accumulated rotation applied to the new
                           iterate (re-orthonormalised by a Newton-Schulz
                           step every 4 calls); same result to rounding,
                           fewer sweeps.  Windows whose rows and rotation
                           fit in LDS together (about min(m,n) * max(m,n)
                           <= 18k) run it in LDS; larger ones run the tiled
                           Jacobi through device memory with the rotation
                           rows staged beside the Jacobi rows (windows that
                           would fit LDS without the rotation take the tiled
                           layout for this).
                           2: as 1, with the start product formed from
                           bfloat16 operands on the matrix cores (FP32
                           accumulation), then refined: the product is
                           recomputed in FP32 with the accumulated rotation
                           and the Jacobi continues (FP32 accuracy).
                           3: bfloat16 start without refinement (precision
                           study; errors of order 1e-3).
                           4: SVD with warm start (Sec. 5, Alg. 2): where
                           mode 1 runs, an SVT may instead take one Cayley
                           step from the previous decomposition (see
                           eps_svd, svdws_every) and shrink its result; the
                           other SVTs are mode 1's, whose decomposition the
                           next step starts from.  An approximation: the
                           shrinkage is not exact after a step.           */
    float jacobi_tol;   /* rotate a pair when |a.b| > tol ||a|| ||b||, with
                           tol = min(cap, max(1e-7, eps2 / (10 mu))) in the
                           inner loop (the SVT's rounding enters Cond2
                           multiplied by mu, up to ~1e3 on large windows) and
                           tol = cap elsewhere; cap = jacobi_tol for rows of
                           up to 256 floats (max(m, n)), jacobi_tol
                           sqrt(256 / max(m, n)) for longer rows; default
                           1e-6                                              */
    int max_sweeps;     /* Jacobi sweep cap, default 40                       */
    int pyramid_levels; /* 1 (default): solve the window as given.  L in 2..4:
                           solve coarse to fine over L levels; level l has the
                           image blurred by the binomial [1 4 6 4 1]/16
                           (borders clamped) and sampled at every second pixel
                           l times, a ceil(m/2^l) x ceil(n/2^l) window, and
                           starts cold from the coarser level's transform
                           conjugated by diag(2, 2, 1).  Not in the paper.     */
    int graph_inner;    /* plain path only: 0 (default) launches the inner
                           iterations one by one; K in 1..256 runs them as
                           replays of a HIP graph of K captured iterations
                           (one stop-flag read per replay).  Same results.   */
    double eps_obj;     /* second outer stop (Alg. 1 "while not converged"):
                           from the second outer iteration of a level on,
                           stop when |f_i - f_{i-1}| < eps_obj f_{i-1} with
                           f = ||A||_* + lambda ||E||_1.  0 (default): off,
                           only ||Delta tau|| < eps_outer and max_outer stop.
                           Not applied by the RASL entry point.              */
    double eps_svd;     /* svt_mode 4: take the Cayley step when
                           ||M_k - M_prev||_F < eps_svd ||M_k||_F (M_prev:
                           the matrix of the previous SVT; the norm and the
                           relative scale are readings), default 1e-3      */
    int svdws_every;    /* svt_mode 4: 0 (default) uses the eps_svd rule;
                           K > 0 replaces it by a fixed schedule: a full SVD
                           in inner iterations 0, K, 2K, ... of each inner
                           loop, the Cayley step in the others (a step with
                           f''(0) <= 0 or a singular system falls back to
                           the full SVD in either rule)                     */
    int reserved_params;
} tilt_params;

/* One window of one image.  The window is given by an initial transform
 * (the problem statement of Eq. TILT_2 starts from D o tau0), either
 * directly (init = 0: tau0) or as the quadrilateral the m x n grid covers
 * in the image (init = 1: quad, mapped as by tilt_tau_from_quad; tau0 is
 * then ignored). */
typedef struct {
    const float* image;     /* host (tilt_solve) or device (batch) pointer    */
    int height, width;
    long long row_stride;   /* elements between rows, >= width                */
    int m, n;               /* rectified rows, columns (>= 2 each)            */
    int model;              /* TILT_AFFINE or TILT_PROJECTIVE                 */
    int init;               /* 0: start from tau0; 1: from quad               */
    double tau0[9];         /* initial pixel homography (init = 0)            */
    double quad[8];         /* window corners TL, TR, BR, BL as (x, y) image
                               pixels (init = 1)                              */
} tilt_problem;

/* Work counters of one solve (used for roofline accounting). */
typedef struct {
    long long inner_iters;      /* LADMAP iterations                          */
    long long svt_calls;        /* singular value decompositions              */
    long long jacobi_sweeps;    /* Jacobi sweeps over all SVDs                */
    long long jacobi_pairs;     /* column pairs examined                      */
    long long jacobi_rotations; /* column pairs rotated                       */
    long long recon_rows;       /* sum over SVDs of singular values kept      */
    long long svdws_steps;      /* svt_mode 4: SVTs done by a Cayley step     */
} tilt_counters;

typedef struct {
    double tau[9];          /* final pixel homography                         */
    float* A;               /* out: m*n, caller-owned; may be NULL            */
    float* E;               /* out: m*n, caller-owned; may be NULL            */
    int outer_iters;
    int inner_iters_total;
    int svt_rank;           /* #singular values of the last M above 1/mu      */
    int status;
    int rank;               /* numerical rank of A: #{sigma_i(A) >
                               1e-3 sigma_1(A)} (FP32 singular values of the
                               last SVT)                                      */
    int reserved;
    double objective;       /* ||A||_* + lambda ||E||_1 of the returned A, E  */
    double mu;              /* penalty at the end of the last inner loop      */
    double cond1, cond2;    /* last values of the Cond1 / Cond2 quantities    */
    double dtau_norm;       /* ||Delta tau||_2 of the last outer iteration    */
    double solve_ms;        /* device time from the start to the end of this
                               patch's solve (device wall clock)              */
    double done_ms;         /* device time from the start of the first patch
                               of the call to the end of this one             */
    tilt_counters counters;
} tilt_result;

/* Fill *p with the defaults listed above. */
void tilt_default_params(tilt_params* p);

/* Human-readable status. */
const char* tilt_status_string(int status);

/* Library version string. */
const char* tilt_version(void);

/* Text of the last HIP runtime error seen by this thread inside the
 * library ("" if none); valid until the next failing call. */
const char* tilt_last_error(void);

/* Homography that maps the centred m x n grid onto a quadrilateral given
 * by its corners TL, TR, BR, BL as (x, y) image pixels (8 doubles).  For
 * TILT_AFFINE the quad must be a parallelogram (the TL, TR, BL corners are
 * used).  Returns TILT_ERR_ARG for degenerate quads. */
int tilt_tau_from_quad(const double quad[8], int m, int n, int model, double tau_out[9]);

/* Plain single-patch path: host pointers in and out, synchronous, on the
 * current device.  Runs Alg. 1 step by step with one kernel per step and one
 * device-to-host read of the stop flags per inner iteration; when the
 * window's SVT does not fit LDS, each round of the tiled Jacobi runs on many
 * workgroups (same results as the batched path).  Allocates and frees its
 * own device memory. */
int tilt_solve(const tilt_problem* prob, const tilt_params* prm, tilt_result* res);

/* ------------------------------------------------------------------------
 * Contexts, batches and serving.
 * ---------------------------------------------------------------------- */
typedef struct tilt_ctx tilt_ctx;

/* Create a context on `device` (HIP ordinal).  hbm_budget_bytes bounds the
 * device workspace the context may hold (0 = 1/2 of free memory). */
int tilt_ctx_create(tilt_ctx** ctx, int device, size_t hbm_budget_bytes);
int tilt_ctx_destroy(tilt_ctx* ctx);

/* Duration in milliseconds of the last fused batch kernel launched through
 * this context, measured with HIP events recorded around the launch on its
 * stream (0 if none). */
int tilt_ctx_last_kernel_ms(tilt_ctx* ctx, double* ms);

/* Progress of the fused kernel that tilt_solve_batch is running on this
 * context, for callers that watch a long batch from another thread:
 * *finished of *total requests are done (both 0 when no fused launch is in
 * flight).  Reads one word of device memory on a stream of its own, so it
 * neither waits for nor delays the batch. */
int tilt_ctx_progress(tilt_ctx* ctx, int* finished, int* total);

/* Bytes of device workspace one problem needs (for admission control), for
 * a single pyramid level and svt_mode 0-3: the larger of the cold and the
 * warm-started layout.  svt_mode 4 adds, where it runs (windows whose
 * warm-started SVT fits LDS), the region of the SVD with warm start: about
 * 4 (13 m n + 14 min(m,n)^2) bytes. */
size_t tilt_workspace_bytes(const tilt_problem* prob);

/* Batched path: `count` problems whose image pointers are DEVICE pointers
 * and whose results' A/E pointers are DEVICE pointers (or NULL).  Runs one
 * fused persistent kernel in which every workgroup solves whole patches
 * from a work queue.  `hip_stream` is a hipStream_t (NULL = default
 * stream).  Returns after the results are on the host (the stream is
 * synchronised).  Per-patch results equal those of tilt_solve. */
int tilt_solve_batch(tilt_ctx* ctx, const tilt_problem* probs, int count,
                     const tilt_params* prm, tilt_result* results, void* hip_stream);

/* Like tilt_solve_batch but forces the step-by-step (plain) kernels for
 * every patch in turn.  Same results, for timing comparisons. */
int tilt_solve_batch_plain(tilt_ctx* ctx, const tilt_problem* probs, int count,
                           const tilt_params* prm, tilt_result* results, void* hip_stream);

/* ------------------------------------------------------------------------
 * Serving (continuous batching).  Requests are admitted while earlier ones
 * are still running: a persistent kernel (one workgroup per compute unit)
 * claims each published request as soon as a workgroup is free, so a
 * request never waits for a batch to fill or drain.  Workspaces come from a
 * device arena owned by the context (min(budget, 8 GiB)); a request that
 * does not fit waits on the host until an earlier one is polled.
 *
 * tilt_submit: validates and queues one problem (image: DEVICE pointer that
 * must stay valid until the request is finished).  A_out / E_out: DEVICE
 * pointers (m x n row-major) or NULL, written when the request finishes.
 * On success *ticket identifies the request.  Argument errors (including
 * TILT_ERR_TOO_LARGE) are returned here and no ticket is issued; a device
 * error while admitting queued requests (TILT_ERR_DEVICE) comes after the
 * request was queued: *ticket is then set and the request can be polled.
 *
 * tilt_poll: TILT_PENDING while the request runs; otherwise fills *res
 * (A/E fields untouched), releases the request and returns its status (a
 * device error while then admitting queued requests is left in
 * tilt_last_error and reported by the next submit or poll).
 * Polling also admits queued requests and restarts the kernel when it has
 * exited after being idle (100 ms without work), so a caller waiting for
 * results must keep polling.  TILT_ERR_NOT_FOUND for unknown or already
 * collected tickets.
 *
 * tilt_serve_stop: waits until every published request has finished,
 * then stops the kernel (requests still queued on the host stay queued;
 * the next submit or poll restarts it).  tilt_ctx_destroy stops it too.
 * Calls on one context are serialised by a lock.
 * ---------------------------------------------------------------------- */
int tilt_submit(tilt_ctx* ctx, const tilt_problem* prob, const tilt_params* prm, float* A_out, float* E_out,
                unsigned long long* ticket);
int tilt_poll(tilt_ctx* ctx, unsigned long long ticket, tilt_result* res);
int tilt_serve_stop(tilt_ctx* ctx);

/* ------------------------------------------------------------------------
 * Components of the hot path, exposed for checking and benchmarking.
 * All pointers are DEVICE pointers unless stated; calls synchronise the
 * stream before returning.
 * ---------------------------------------------------------------------- */

/* Singular value shrinkage A_i = S_{eps_i}(M_i) = U T_eps(Sigma) V^T
 * (Eqs. A_1 and S_operator) of `count` m x n row-major matrices stored back
 * to back (M + i*m*n), by the same one-sided Jacobi used inside the solver.
 * eps: HOST array of count non-negative floats.  sigma (count*min(m, n),
 * unsorted) may be NULL.  ranks (HOST, count) receives #{sigma > eps_i} and
 * counters (HOST) the summed work counters; both may be NULL.  Only the
 * Jacobi fields of prm are read. */
int tilt_svt_batch(tilt_ctx* ctx, const float* M, float* A, float* sigma, int count, int m, int n,
                   const float* eps, const tilt_params* prm, int* ranks, tilt_counters* counters,
                   void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * tilt_svt_batch without a context and without any device allocation.  The
 * same shrinkage by the same kernels; every device buffer beyond the
 * caller's inputs and outputs (job table, per-matrix work counters and
 * ranks, per-matrix working planes) comes from one fixed array of
 * TILT_SVT_NOALLOC_BYTES in the library, one per GPU, held until the
 * process ends.  Runs on the current device and on `hip_stream`; other
 * arguments as in tilt_svt_batch (eps, ranks and counters are HOST arrays).
 * Per matrix the batch needs 8 min(m,n) ldg bytes (ldg = max(m,n) rounded
 * up to 4), plus 4 ncp ldg bytes when the shape's SVT is tiled (ncp: its
 * rows rounded up to whole super-blocks), plus about 64 bytes; a batch that
 * needs more than the array returns TILT_ERR_TOO_LARGE before any device
 * work.  Every call on a GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU race; calls in sequence
 * (one stream, or synchronised) are safe.  Synchronous. */
#define TILT_SVT_NOALLOC_BYTES ((size_t)64 << 20)
int tilt_svt_batch_noalloc(const float* M, float* A, float* sigma, int count, int m, int n,
                           const float* eps, const tilt_params* prm, int* ranks, tilt_counters* counters,
                           void* hip_stream);

/* SVD with warm start (Sec. 5, Alg. 2, with the derivatives of Appendix A):
 * one Cayley step per matrix, for `count` matrices of one shape m x n
 * (m >= n, n <= 256, m <= 4096), DEVICE arrays back to back, row-major:
 * the previous decomposition U (m x n, orthonormal columns), S (n), V
 * (n x n, orthogonal; M ~ U diag(S) V^T) and the next matrix M (m x n).
 * The step searches U(t) = (I + t/2 P_U)^{-1} (I - t/2 P_U) U, S(t) =
 * S - t P_S, V(t) = (I + t/2 P_V)^{-1} (I - t/2 P_V) V along the projected
 * gradients of 1/2 ||M - U S V^T||_F^2 (Eqs. projected_gradient1-3) and
 * takes t = -f'(0)/f''(0) of the model of Eq. ft.  P_U (m x m, rank <= 2n)
 * is never formed; its Cayley factor goes through the Woodbury identity
 * (a 2n x 2n solve).  Outputs U_out, S_out, V_out (DEVICE, the input
 * shapes) and, unless A_out is NULL, A_out = U(t) T_eps(S(t)) V(t)^T with
 * the signed soft threshold eps[i] (HOST array).  HOST arrays t_out, f0_out
 * (f(0)), ft_out (f(t)) and status may be NULL.  status[i]: 0 = step taken;
 * 1 = f''(0) <= 0, no step (outputs = inputs; Alg. 2's caller computes a
 * full SVD instead, as it does when ||M - M_prev|| >= eps_svd); -4 = a
 * singular system.  Alg. 2's switch between this step and a full SVD is the
 * caller's.  Synchronous; returns the worst error status (warnings are not
 * reported in the return value). */
int tilt_svdws_batch(tilt_ctx* ctx, int count, int m, int n, const float* U, const float* S, const float* V,
                     const float* M, float* U_out, float* S_out, float* V_out, float* A_out, const float* eps,
                     double* t_out, double* f0_out, double* ft_out, int* status, void* hip_stream);

/* Alg. 1 Step 1 on its own: the normalised warp D o tau / ||D o tau||_F
 * (I_out: count x m x n) and the Jacobian of the normalised warp w.r.t.
 * the p entries of tau in scaled coordinates (J_out: count x p x m x n,
 * parameter-major; order h11 h12 h13 h21 h22 h23 [h31 h32]).  The scaled
 * coordinates are those of the window given by probs[i].tau0; taus (HOST,
 * count x 9) are the pixel homographies at which to evaluate.  All
 * problems must share m, n and model. */
int tilt_warp_jacobian(tilt_ctx* ctx, const tilt_problem* probs, const double* taus, int count,
                       float* I_out, float* J_out, void* hip_stream);

/* The LADMAP inner loop alone (Sec. 3.2 in the form of Sec. 4.2; the
 * setting of Table 1): for `count` problems of one shape,
 *     min ||A||_* + lambda ||E||_1  s.t.  I + J dtau = A + E
 * with I (count x m x n, row-major) and J (count x p x m x n, one m x n
 * plane per column) given as DEVICE arrays, 1 <= p <= 5.  No
 * normalisation and no extra constraints; starts from A = I, E = Y = 0
 * with mu_0 from params (<= 0: 1.25/||I||_2).  A, E (count x m x n,
 * DEVICE) may be NULL.  Fills inner_iters_total, objective, mu, cond1,
 * cond2, svt_rank, status, solve_ms and the counters of results[i]; tau is
 * zero.  max(m, n) <= 2048, min(m, n) <= 1024; pyramid_levels must be 1.
 * When the SVT does not fit LDS and count <= (compute units) / 8, each
 * Jacobi round of a problem runs on many workgroups (one per super-block
 * pair, one launch per round) instead of one workgroup per problem. */
int tilt_inner_batch(tilt_ctx* ctx, const float* I, const float* J, int count, int m, int n, int p,
                     const tilt_params* prm, float* A, float* E, tilt_result* results, void* hip_stream);

/* ------------------------------------------------------------------------
 * Jacobi layout tuning.  The layout of the LDS-resident Jacobi (rows per
 * block, lanes per row pair; the float4 chunks per lane, and for two-row
 * blocks of 8 or 16 lanes up to 2 single floats per lane that stand in for
 * a mostly empty last chunk, follow from the row length) is chosen by a
 * cost model unless a measured entry applies: a
 * window whose min(m,n) and max(m,n) are both within a factor 1.5 of a
 * tuned shape uses the layout measured for the nearest one (if valid for
 * its row length).  The table is process-wide; calls are thread-safe and
 * affect problems planned afterwards.
 * ---------------------------------------------------------------------- */

/* Valid layouts for an m x n window: writes up to max_count (rows per block,
 * lanes per pair) pairs and returns how many exist (0 for tiled shapes). */
int tilt_svt_layouts(int m, int n, int* bs, int* lpp, int max_count);
/* Record the measured best layout for an m x n window. */
int tilt_tune_set(int m, int n, int bs, int lpp);
/* Forget all measured layouts (back to the cost model). */
int tilt_tune_clear(void);
/* The layout an m x n window's SVT runs with, as planned now (table and
 * cost model): out[0..4] = rows per block, lanes per pair, float4 chunks
 * per lane, single floats per lane, and 1 if the matrix is tiled through
 * device memory (then out[0..3] describe the staged super-block pair).
 * Host-only, no device work.  TILT_ERR_ARG for a null out or m, n < 1;
 * TILT_ERR_TOO_LARGE if no SVT plan exists for the shape. */
int tilt_svt_layout(int m, int n, int* out);

/* ------------------------------------------------------------------------
 * Machine peaks for the rooflines (not part of the method): one probe
 * kernel, built with the solver's compiler flags, runs on the stream and
 * *ms_out receives its duration (HIP events), *work_out the work it did.
 *   kind 0: HBM stream copy of `bytes` (rounded down to 16) from src to dst
 *           (DEVICE buffers of at least `bytes` each); work = bytes read +
 *           written.
 *   kind 1: LDS 16-byte reads (consecutive lanes, no bank conflicts), iters
 *           x 8 per thread; work = LDS bytes read.
 *   kind 2: FP32 vector FMA (8 independent chains per lane, iters steps);
 *           work = flops.
 *   kind 3: FP32 matrix-core MFMA 16x16x4 (4 accumulators per wavefront,
 *           iters steps); work = flops.
 * Kinds 1-3 run 8 workgroups of 256 threads per compute unit and write one
 * 4-byte word per thread to dst, which must hold `bytes` >= that many
 * words; src is unused.  Synchronous.  TILT_ERR_ARG for a bad kind, null
 * pointers, iters < 1 (kinds 1-3) or a dst too small.
 * ---------------------------------------------------------------------- */
int tilt_peak_probe(int kind, const void* src, void* dst, size_t bytes, int iters, double* ms_out,
                    double* work_out, void* hip_stream);

/* Pyramid levels 1..levels-1 of one image (DEVICE pointers), as used when
 * pyramid_levels = levels: level l (ceil(H/2^l) x ceil(W/2^l), row-major,
 * contiguous) follows level l-1 in `out`.  levels in 2..4. */
int tilt_pyramid(tilt_ctx* ctx, const float* image, int height, int width, long long row_stride, float* out,
                 int levels, void* hip_stream);

/* ------------------------------------------------------------------------
 * RASL variant.  The paper (Sec. 1, on RASL) notes that TILT and RASL share
 * one model and differ only in the data matrix: for RASL it holds several
 * images, one per column.  Here column k is the m x n window of image k
 * warped by its own transform tau_k and normalised to unit norm; its
 * Jacobian depends on tau_k alone, so J_perp acts on every column
 * separately, and Alg. 1 runs unchanged otherwise (Sec. 4.2 inner loop,
 * Delta tau_k = (J_k^T J_k)^{-1} J_k^T (a_k + e_k - d_k)).  No extra
 * constraints are put on the transforms; lambda <= 0 selects
 * 1/sqrt(max(m n, count)); the outer loop stops when the norm of all
 * Delta tau_k together is below eps_outer.
 * ---------------------------------------------------------------------- */
typedef struct {
    const float* images;     /* DEVICE: `count` images, image k at images + k * image_stride */
    long long image_stride;  /* floats from one image to the next                          */
    int height, width;       /* size of every image (>= 2 x 2)                             */
    long long row_stride;    /* floats from one image row to the next (>= width)           */
    int count;               /* images = columns of the data matrix, 2 <= count < m n      */
    int m, n;                /* common rectified window, m n <= 2048                       */
    int model;               /* TILT_AFFINE or TILT_PROJECTIVE                             */
    const double* tau0;      /* HOST: count row-major 3x3 homographies, centred window
                                pixel (u, v, 1) -> image pixel (x, y, 1)                    */
} tilt_rasl_problem;

typedef struct {
    double* tau;             /* HOST, caller-allocated count x 9: the final transforms     */
    float* A;                /* DEVICE, caller-allocated count x m x n (window k row-major
                                at k m n), or NULL                                         */
    float* E;                /* same layout, or NULL                                       */
    double objective;        /* ||A||_* + lambda ||E||_1 of the last inner loop            */
    int outer_iters, inner_iters_total;
    int svt_rank;            /* singular values of the last SVT argument above 1/mu        */
    int status;              /* TILT_OK, TILT_WARN_MAXITER or an error                     */
    double solve_ms;         /* device wall-clock time of this solve                       */
    tilt_counters counters;  /* work counters of this solve                                */
} tilt_rasl_result;

/* Solve `count` independent RASL problems in one fused kernel (one
 * workgroup per problem, work queue).  Inputs and A/E are device memory;
 * tau0 and tau are host memory.  `prm->svt_mode` must be 0 and
 * `prm->pyramid_levels` 1.  TILT_ERR_ARG for invalid shapes or transforms,
 * TILT_ERR_TOO_LARGE when m n exceeds 2048 or the count x m n matrix does not
 * fit the SVT; per-problem failures are in res[k].status and the call
 * returns the worst status.  The stream is synchronised before returning. */
int tilt_rasl_solve_batch(tilt_ctx* ctx, const tilt_rasl_problem* probs, int count, const tilt_params* prm,
                          tilt_rasl_result* res, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* TILT_H */
