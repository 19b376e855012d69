/*
 * cpqr.h -- C ABI of the MI355X (gfx950) CP-ALS-QR library (libcpqr.so).
 *
 * The library computes a rank-R CP decomposition of a dense order-N tensor
 * with the QR-based alternating least squares of arXiv 2503.18759:
 * Algorithm 2 (CP-ALS-QR) and Algorithm 3 (ALS-QR-BRE), with the TTM chain
 * organised by no tree, the standard dimension tree, or the restructured
 * dimension tree of Section 3.1, and the customised Q0 extrapolation of
 * eq. (19).
 *
 * Conventions shared by every entry point
 *  - Every function returns a cpqr_status: 0 on success, a negative code on
 *    failure.  No C++ exception crosses the ABI.
 *  - Dense tensors are column-major with mode 1 fastest: element
 *    (i_1, ..., i_N) sits at i_1 + I_1 (i_2 + I_2 (i_3 + ...)), the
 *    unfolding convention of Section 2.1.  Matrices are column-major.
 *  - "device" pointers are HIP device allocations (for example torch CUDA
 *    tensors on ROCm); "host" pointers are ordinary CPU memory.
 *  - Validation of sizes and pointers happens before any device work; on a
 *    validation error nothing is launched and outputs are untouched.
 *  - A handle is bound to one device and one HIP stream.  Calls on a handle
 *    are synchronous with respect to the host (they return after results
 *    are copied out) and must not be made concurrently from several threads.
 */
#ifndef CPQR_H
#define CPQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPQR_OK = 0,
  CPQR_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad enum) */
  CPQR_EUNSUPPORTED = -2, /* valid but outside what this build handles (see limits) */
  CPQR_ENOMEM = -3,       /* device allocation failed */
  CPQR_EHIP = -4,         /* a HIP runtime call failed; see cpqr_last_error */
  CPQR_ERANKDEF = -5,     /* a column norm (lambda_r), a diagonal of R0 or R_n, or a diagonal of an
                             initial factor's R is zero or at most 1e-13 times the largest of its
                             set (numerically dependent columns, e.g. duplicate initial columns) */
  CPQR_ENONFINITE = -6    /* a NaN or Inf appeared in the fit or in lambda */
} cpqr_status;

/* TTM organisation (Section 3.1 / 3.4).  NONE contracts each leaf directly
 * from X; STANDARD is the dimension tree of Figure 1 / Tables 1 and 4;
 * RESTRUCTURED is the restructured dimension tree (Tables 2 and 5), which
 * also permutes the per-sweep update order. */
typedef enum { CPQR_TREE_NONE = 0, CPQR_TREE_STANDARD = 1, CPQR_TREE_RESTRUCTURED = 2 } cpqr_tree;

/* Q0 extrapolation (Section 3.2, eq. (19), Algorithm 3).  OFF is beta = 0
 * (ALS-QR-BR); PAPER activates beta once the fit change drops below
 * switch_delta and picks it from the fit level (Section 4.3).  LEARNED (a
 * feature of this library, not of the paper) takes beta from the MLP in
 * cpqr_options.mlp_weights after sweep 2 and applies it from sweep 3 through
 * the same eq. (19) update.  The state after sweep 2 is the checkpoint, with
 * its explicit fit 1 - ||X - K|| / ||X|| (float64).  Checks follow after 4
 * sweeps, then after gaps that double (8, 16, ...), at the last sweep of the
 * run and at a tolerance stop: the explicit fit, with lambda divided by
 * 1 + (1 - alpha) beta (the factor by which eq. (19) scales an update at a
 * fixed point), must exceed the checkpoint's, and the state becomes the new
 * checkpoint; otherwise the checkpoint is restored (factors, Q0 of its sweep,
 * the intermediates live across it), beta becomes the paper's table value
 * for the checkpoint's fit, and the sweeps since the checkpoint run again
 * with it, with no further checks (the MLP is not consulted again). */
typedef enum { CPQR_EXTRAP_OFF = 0, CPQR_EXTRAP_PAPER = 1, CPQR_EXTRAP_LEARNED = 2 } cpqr_extrap;

/* Learned-extrapolation MLP: CPQR_MLP_FEATURES inputs -> CPQR_MLP_HIDDEN tanh
 * units -> one linear output y = u, the momentum share u = g beta / (1 + g beta)
 * with g = 0.9: beta = u / (g (1 - u)) for u clamped to [0, 27/28]
 * (beta in [0, 30]).
 * Parameters (float32, CPQR_MLP_PARAMS): W1 (HIDDEN x FEATURES, row-major),
 * b1 (HIDDEN), w2 (HIDDEN), b2 (1).  Features after sweep 2 (fits f1, f2 of
 * sweeps 1 and 2, order N, rank R, mode sizes I_n):
 *   [f1, f2, 10 (f2 - f1), log10(max(1 - f2, 1e-12)) / 4, N / 5, R / 16,
 *    log2(mean I_n) / 8, R / min I_n]. */
#define CPQR_MLP_FEATURES 8
#define CPQR_MLP_HIDDEN 64
#define CPQR_MLP_PARAMS (CPQR_MLP_HIDDEN * CPQR_MLP_FEATURES + 2 * CPQR_MLP_HIDDEN + 1)

/* Arithmetic of the TTM chain.  FP64 needs a float64 tensor; FP32 and
 * BF16X3 need a float32 tensor.  BF16X3 computes each TTM product as
 * x_hi q_hi + x_hi q_lo + x_lo q_hi on bf16 matrix cores with float32
 * accumulation.  The QRs, the triangular solves, Y_(n) Q0 and the fit are
 * float64 in every mode. */
typedef enum { CPQR_PREC_FP64 = 0, CPQR_PREC_FP32 = 1, CPQR_PREC_BF16X3 = 2 } cpqr_prec;

typedef enum { CPQR_DTYPE_F64 = 0, CPQR_DTYPE_F32 = 1 } cpqr_dtype;

/* Option flags. */
#define CPQR_FLAG_EXPLICIT_FIT 0x1u  /* also compute 1 - ||X - K|| / ||X|| explicitly at the end */
#define CPQR_FLAG_TIME_KERNELS 0x2u  /* time every level-1 TTM (the TTM that reads X) with HIP events:
                                        kernels launch one by one, and each level-1 TTM runs as a graph
                                        of 8 back-to-back launches (it is idempotent) between two events */
#define CPQR_FLAG_NO_GRAPH     0x4u  /* launch kernels one by one instead of replaying HIP graphs */
#define CPQR_FLAG_DENSE_ZQR    0x8u  /* factor Z_n by the dense two-level TSQR even where the
                                        one-workgroup staircase QR (Z_n of at most 1024 rows) or
                                        the nested two-factor QR (order >= 4) applies; for
                                        comparison */
#define CPQR_FLAG_TIME_PHASES  0x10u /* fill cpqr_result.phase_seconds: kernels launch one by one
                                        (no graphs) with HIP events between kernel groups, and the
                                        host waits after every sweep; excludes TIME_KERNELS */
#define CPQR_FLAG_CLOSING_PLAIN 0x20u /* the last sweep (sweep `iters`) runs without extrapolation
                                        (beta = 0): at a fixed point eq. (19) scales every update
                                        by 1 + (1 - alpha) beta, which lambda carries; a plain
                                        sweep gives the extrapolated factors their own lambda */

typedef struct cpqr_handle cpqr_handle;

/* Create a handle on `device` that launches on `hip_stream` (a hipStream_t;
 * NULL = the default stream).  The handle owns all device workspace, which
 * is allocated on first use, grown on demand and freed by cpqr_destroy. */
cpqr_status cpqr_create(cpqr_handle **handle, int device, void *hip_stream);
cpqr_status cpqr_destroy(cpqr_handle *handle);

/* Message describing the last error on this handle ("" if none).  The
 * string is owned by the handle.  With handle == NULL: the message of the
 * last failed cpqr_qr_noalloc call on the calling host thread. */
const char *cpqr_last_error(const cpqr_handle *handle);
/* Static name of a status code. */
const char *cpqr_status_string(int status);

typedef struct {
  int order;            /* 3 <= N <= 7 (N = 2 is accepted with CPQR_TREE_NONE) */
  const int64_t *dims;  /* host, N mode sizes I_1..I_N, each >= 1 */
  int dtype;            /* cpqr_dtype */
  const void *data;     /* device, prod(dims) elements, column-major (mode 1 fastest) */
} cpqr_tensor;

typedef struct {
  int tree;             /* cpqr_tree */
  int extrapolate;      /* cpqr_extrap */
  int prec;             /* cpqr_prec */
  int iters;            /* number of sweeps m (Algorithm 2/3 input), >= 1 */
  double tol;           /* stop when |fit_k - fit_{k-1}| < tol; 0 = run all sweeps */
  double alpha;         /* eq. (19) alpha; the paper uses 0.1 */
  double switch_delta;  /* activation threshold on the fit change; the paper uses 0.03 */
  double fixed_beta;    /* if > 0 with CPQR_EXTRAP_PAPER: use this beta from sweep 2 on instead of the rule */
  const double *const *init_factors; /* host, N pointers to I_n x R column-major float64 initial factors,
                                        or NULL: seeded N(0,1) factors (see `seed`) */
  unsigned flags;       /* CPQR_FLAG_* */
  const float *mlp_weights; /* host, CPQR_MLP_PARAMS floats; required with CPQR_EXTRAP_LEARNED, else ignored */
  const double *beta_schedule; /* host, `iters` values or NULL.  With CPQR_EXTRAP_PAPER: sweep k+1 uses
                                  beta = beta_schedule[k] (k >= 1; entry 0 is unused since sweep 1 has
                                  no previous Q0), overriding the rule and fixed_beta.  Used to label the
                                  training data of the learned extrapolation. */
  uint64_t seed;        /* with init_factors == NULL: entry e of the initial factors (modes in order,
                           each I_n x R column-major, e counting across modes) is the Box-Muller
                           normal sqrt(-2 ln u_{2e}) cos(2 pi u_{2e+1}), u_j = ((z_j >> 11) + 0.5) 2^-53,
                           z_j = output j (0-based) of SplitMix64 seeded with `seed`
                           (z_j = mix64(seed + (j + 1) 0x9E3779B97F4A7C15), mix64 the finaliser of
                           Steele, Lea and Flood, OOPSLA 2014); ignored otherwise */
} cpqr_options;

typedef struct {
  double *const *factors;  /* host, N caller-owned I_n x R float64 outputs (unit-norm columns), or NULL */
  double *lambda;          /* host, R weights, or NULL */
  double *fit_history;     /* host, `iters` per-sweep fits (Section 4.1 formula), or NULL */
  int *sweep_orders;       /* host, iters x N 0-based update orders, or NULL */
  double fit;              /* fit after the last sweep (Section 4.1 formula) */
  double fit_explicit;     /* explicit 1 - ||X-K||/||X|| if CPQR_FLAG_EXPLICIT_FIT, else NaN */
  int sweeps_done;
  double beta;             /* extrapolation weight in force at the end (0 if never active) */
  int beta_sweep;          /* sweep after which beta was activated (0 if never) */
  double ttm_flops;        /* TTM flops executed (2 |input| R per TTM) */
  double ttm_bytes;        /* TTM algorithmic bytes (input read once + output written once) */
  double seconds;          /* device wall time of the sweep loop */
  double l1_ttm_seconds;   /* with CPQR_FLAG_TIME_KERNELS: summed per-launch duration of the level-1 TTMs */
  int l1_ttm_launches;     /* number of level-1 TTMs timed */
  double l1_ttm_bytes;     /* algorithmic bytes of one level-1 TTM per launch (averaged) */
  double l1_ttm_flops;     /* flops of one level-1 TTM per launch (averaged) */
  double beta_learned;     /* CPQR_EXTRAP_LEARNED: the MLP's beta (0 otherwise) */
  int learned_fallback_sweep; /* CPQR_EXTRAP_LEARNED: sweep whose rejection switched to the paper's beta (0 if none) */
  double phase_seconds[5]; /* with CPQR_FLAG_TIME_PHASES (else 0): summed device time of the sweeps in the
                              five categories of the time breakdown of Section 4.2:
                              [0] TTM (every TTM of the tree),
                              [1] QR (the factor-QR kernels, which also carry the fused triangular
                                  solve, normalisation, fit and beta rule of the update),
                              [2] computation of Q0 (the QR of Z_n),
                              [3] application of Q0 (Y_(n) [Q0 | Q0^{k-1}] and its reduction),
                              [4] other (the gaps between kernel groups: launch and event latency) */
  double *const *q_factors; /* host, N caller-owned I_n x R float64 outputs, or NULL: the explicit Q_n of
                               the last factor QRs as the TTMs used them (float32 values for FP32 and
                               BF16X3, widened exactly), for the orthonormality report ||Q_n^T Q_n - I||;
                               a mode with I_n < R has zero columns beyond I_n */
} cpqr_result;

/*
 * cpqr_als_qr -- CP-ALS-QR / ALS-QR-BR / ALS-QR-BRE (Algorithms 2 and 3).
 * Inputs: tensor X (device), rank R, options (iteration count, stopping
 * tolerance, tree, extrapolation, precision, initial factors).  Outputs
 * (host, caller-owned): factor matrices with unit-norm columns, lambda, the
 * per-sweep fit history and update orders, and the final fit.
 * A mode may be smaller than the rank: its factor gets the compact QR with
 * min(I_n, R) reflectors (Q_n is I_n x I_n, R_n upper trapezoidal), held on
 * the device zero-padded to I_n x R and R x R.  Every Z_n then has
 * prod_{k != n} min(I_k, R) nonzero rows, which must be at least R
 * (otherwise P^(n) cannot have full column rank: CPQR_EUNSUPPORTED).
 * A mode of more than 512 rows has its factor QR done by the two-level
 * TSQR (solve and normalisation stream the rows through one workgroup);
 * its size must fit that TSQR: I_n <= 8192 at R <= 32, 65536 at R <= 16,
 * 524288 at R <= 8 (CPQR_EUNSUPPORTED otherwise; the batched entry point
 * keeps I_n <= 512).
 * Limits of this build: 1 <= R <= 32, and the order N at most 4 for
 * 17 <= R <= 32, 6 for 9 <= R <= 16 and 7 for R <= 8 (Z_n of order N >= 4
 * is factored by N - 2 nested two-factor QRs of R^2 rows, Section 2.4's
 * QR of the Khatri-Rao product taken level by level).  With
 * CPQR_FLAG_DENSE_ZQR, and for every problem of cpqr_als_qr_batched, Z_n
 * (R^(N-1) x R, including the zero rows of padded modes) must also fit a
 * two-level TSQR: ceil(R^(N-1) / B) * R <= B with B = 2048, 1024, 512 rows
 * for R <= 8, 16, 32 (for example 40^5 at R = 16 and 256^3 at R = 32 fit).
 * On a runtime error (CPQR_ERANKDEF, CPQR_ENONFINITE, CPQR_EHIP) the outputs
 * are untouched except sweeps_done and fit_history up to the failure.
 */
cpqr_status cpqr_als_qr(cpqr_handle *handle, const cpqr_tensor *X, int rank,
                        const cpqr_options *opts, cpqr_result *result);

/*
 * Step-wise form of cpqr_als_qr.  A session holds one decomposition in
 * progress on the device; cpqr_als_qr is create + sweeps(iters) + result +
 * destroy.  A handle has at most one live session (its workspace is shared).
 *
 * cpqr_session_create -- validate as cpqr_check_args, allocate workspace,
 *   upload and QR-factor the initial factors (Algorithm 2 "Initialize") and
 *   compute ||X||^2.  X must stay allocated and unchanged until the session
 *   is destroyed.  opts->iters is the maximum number of sweeps.  Errors as
 *   cpqr_als_qr, plus CPQR_EINVAL if the handle already has a live session.
 * cpqr_session_sweeps -- enqueue the next `nsweeps` sweeps on the handle's
 *   stream.  Asynchronous unless opts->tol > 0, in which case the fit is read
 *   back after each sweep and the session stops once the tolerance is met
 *   (later calls then do nothing).  CPQR_EINVAL if the total would exceed
 *   opts->iters.
 * cpqr_session_sync -- wait for the enqueued sweeps.
 * cpqr_session_result -- wait, then fill `result` (caller-owned host
 *   buffers, as for cpqr_als_qr) for the sweeps run so far; `seconds` is the
 *   device time since the first cpqr_session_sweeps call.
 * cpqr_session_destroy -- wait and release the session.
 */
typedef struct cpqr_session cpqr_session;
cpqr_status cpqr_session_create(cpqr_handle *handle, const cpqr_tensor *X, int rank,
                                const cpqr_options *opts, cpqr_session **session);
cpqr_status cpqr_session_sweeps(cpqr_session *session, int nsweeps);
cpqr_status cpqr_session_sync(cpqr_session *session);
cpqr_status cpqr_session_result(cpqr_session *session, cpqr_result *result);
cpqr_status cpqr_session_destroy(cpqr_session *session);

/*
 * cpqr_als_qr_batched -- `count` independent decompositions run together
 * (a batching feature of this library, not part of the paper's method: each
 * problem follows Algorithm 2 / 3 exactly as cpqr_als_qr would).  Every sweep
 * of the whole batch is one HIP graph whose kernels each cover all problems
 * (grid dimension = problem); the float32 TTM launches are autotuned (K split
 * across the waves of a workgroup) on the first sweep by timing the
 * candidates into scratch outputs.
 * Xs[t], ranks[t], opts[t], results[t]: the arguments of cpqr_als_qr for
 * problem t (same meaning, layout and ownership).  All problems must share
 * order, tree, extrapolate, prec and iters (alpha, switch_delta and
 * fixed_beta may differ); prec must be CPQR_PREC_FP32 or CPQR_PREC_BF16X3;
 * tol must be 0 (every problem runs exactly `iters` sweeps); extrapolate
 * must be OFF or PAPER.  Violations: CPQR_EINVAL (mixed settings, tol != 0,
 * count < 1) or CPQR_EUNSUPPORTED (FP64, LEARNED).  Each problem is
 * validated as cpqr_check_args; the first failing problem's status is
 * returned and nothing runs.  Runtime errors are reported per problem: the
 * function returns the first non-OK status over t = 0..count-1 after filling
 * every result it can.  Uses the handle's workspace; CPQR_EINVAL if the
 * handle has a live session.
 */
cpqr_status cpqr_als_qr_batched(cpqr_handle *handle, int count, const cpqr_tensor *Xs,
                                const int *ranks, const cpqr_options *opts,
                                cpqr_result *results);

/*
 * MLP of the learned extrapolation (a feature of this library, not of the
 * paper).  Weights, inputs and outputs are host float32 arrays; the
 * arithmetic runs on the device.  x is n x CPQR_MLP_FEATURES row-major.
 * cpqr_mlp_forward -- y[i] = output for row i.
 * cpqr_mlp_grad -- loss = (1/2n) sum_i (y_hat_i - y_i)^2 and its gradient with
 *   respect to the CPQR_MLP_PARAMS weights (same layout).
 * cpqr_mlp_train -- `epochs` passes of Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 *   step size lr) over shuffled mini-batches of `batch` rows (seeded order);
 *   w is updated in place; loss_history (epochs entries, or NULL) receives
 *   the mean-squared loss over all n rows after each epoch.
 * Errors: CPQR_EINVAL for null pointers, n < 1, batch < 1, epochs < 0.
 */
cpqr_status cpqr_mlp_forward(cpqr_handle *handle, const float *w, const float *x, int n, float *y);
cpqr_status cpqr_mlp_grad(cpqr_handle *handle, const float *w, const float *x, const float *y, int n,
                          float *loss, float *grad);
cpqr_status cpqr_mlp_train(cpqr_handle *handle, float *w, const float *x, const float *y, int n,
                           int epochs, int batch, float lr, uint64_t seed, float *loss_history);

/*
 * cpqr_check_args -- host-only: the argument checks that cpqr_als_qr makes
 * before any device work (pointers, sizes, enums, precision/dtype match and
 * the limits of this build).  Returns the status cpqr_als_qr would return
 * for these arguments before launching anything; needs no device.
 */
cpqr_status cpqr_check_args(const cpqr_tensor *X, int rank, const cpqr_options *opts);

/*
 * cpqr_schedule -- host-only: the TTM schedule of `sweeps` sweeps of an
 * order-`order` problem for `tree` (Section 3.1, Tables 1-6).
 *  orders_out : host, sweeps x order ints (0-based mode update order), or NULL.
 *  steps_out  : host, up to max_steps x 3 ints per step: {kind, src_mask, mode}
 *               kind 0 = TTM contracting `mode` of Y{src_mask} (src_mask is
 *               the bitmask of free modes; all bits set = X), kind 1 = mode
 *               update consuming the leaf Y{mode}.  May be NULL.
 *  n_steps    : host, receives the total number of steps.
 *  flops_out  : host, 2^order x order doubles or NULL: coefficient of the
 *               monomial prod_{k in mask} I_k * R^(order-|mask|+1) at index
 *               mask * order + 0 summed over all sweeps (other entries 0).
 * Returns CPQR_EINVAL for order < 2 or > 8, bad tree, sweeps < 1, or when
 * max_steps is too small for steps_out.
 */
cpqr_status cpqr_schedule(int order, int tree, int sweeps, int *orders_out,
                          int *steps_out, int max_steps, int *n_steps,
                          double *flops_out);

/*
 * Tuned TTM launch shapes (not in the paper: an autotuner of this library).
 * The first session or batch that meets a float32 TTM shape times its launch
 * shapes (K split 1/2/4 waves per 64-row output tile, 1 or 2 workgroups per
 * CU) and keeps the fastest in the handle and in a JSON file:
 *   {"format": 1, "device": "<gcnArchName>:<CUs>",
 *    "entries": {"<key>": [ks, wpc], ...}}
 * at $CPQR_TUNE_CACHE, else $XDG_CACHE_HOME/cpqr/ttm_tune.json, else
 * $HOME/.cache/cpqr/ttm_tune.json; CPQR_TUNE_CACHE=off keeps the results in
 * memory.  Entries for another device signature are ignored.
 *
 * cpqr_tune_cache_check -- host-only: parses the text of such a file.
 *  text    : host, NUL-terminated file contents.
 *  device  : host, NUL-terminated device signature ("gfx950:256").
 *  entries : host, receives the number of entries valid for `device` (0 when
 *            the file was written for another device), or NULL.
 * Returns CPQR_OK for a well-formed file, CPQR_EINVAL otherwise (null text or
 * device, syntax errors, unknown fields, shapes outside the candidates).
 */
cpqr_status cpqr_tune_cache_check(const char *text, const char *device, int *entries);

/*
 * cpqr_tune_cache_path -- the file the handle's tuning results go to
 * (empty when persistence is off) and the handle's device signature.
 *  path, device : host buffers of `cap` bytes each (NUL-terminated, truncated
 *                 to fit); either may be NULL.
 * Returns CPQR_EINVAL for a null handle.
 */
cpqr_status cpqr_tune_cache_path(cpqr_handle *handle, char *path, char *device, int cap);

/*
 * cpqr_ttm -- one mode-m product Y = X x_m Q^T (Section 2.1): the tensor
 * `in` (device, dims[0..order-1], column-major) is contracted on mode `mode`
 * (0-based) with Q (device, dims[mode] x R column-major, same precision as
 * the TTM: float64 for FP64, float32 for FP32; for BF16X3 `q` is float32 and
 * is split on the device).  `out` (device) receives the tensor with
 * dims[mode] replaced by R.  in/out element type: float64 for FP64, float32
 * otherwise.  Limits: 1 <= R <= 64, roundup(dims[mode],32) * roundup(R,16) * 4 <= 160 KiB.
 */
cpqr_status cpqr_ttm(cpqr_handle *handle, int prec, int order, const int64_t *dims,
                     int mode, int rank, const void *in, const void *q, void *out);

/*
 * cpqr_qr -- the compact QR of Section 2.4 (the QR of every factor matrix and
 * of Z_n in Algorithm 2) for an M x R float64 matrix held on the device
 * (column-major): A = Q R with Q (device, M x R, orthonormal columns) and R
 * (device, R x R, upper triangular, non-negative diagonal), computed by
 * Householder reflections (two-level TSQR for tall matrices).  A, Q and R
 * are caller-owned; the handle owns the TSQR workspace (allocated on demand).
 * Errors: CPQR_EINVAL for null pointers or R > M, CPQR_EUNSUPPORTED beyond
 * the limits 1 <= R <= 32, M within the two-level TSQR (M <= 2^20 at R <= 8).
 */
cpqr_status cpqr_qr(cpqr_handle *handle, int64_t M, int R, const double *A,
                    double *Q, double *Rout);

/*
 * cpqr_qr_noalloc -- cpqr_qr for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arithmetic and results as cpqr_qr (the same kernels),
 * but no handle: the TSQR scratch lives in a fixed device array of
 * CPQR_QR_NOALLOC_SCRATCH_BYTES per device, held until the process ends, and
 * the call allocates nothing (no hipMalloc/hipFree, no allocating library
 * routine).  Runs on the current device (hipSetDevice) and enqueues on
 * `hip_stream` (a hipStream_t; NULL = the default stream) without
 * synchronising: Q and Rout are ready when the stream reaches the call.
 *  A    : device, M x R float64, column-major (caller-owned, read only).
 *  Q    : device, M x R float64, column-major (caller-owned output).
 *  Rout : device, R x R float64, column-major, upper triangular with a
 *         non-negative diagonal (caller-owned output).
 * All calls on one device share that device's scratch, which keeps the last
 * call's contents: calls that overlap on one device (several streams or
 * host threads) race and must be serialised by the caller.
 * Errors (checked before any device work; message via cpqr_last_error(NULL)):
 * CPQR_EINVAL for null pointers or R > M; CPQR_EUNSUPPORTED for R > 32,
 * sizes beyond the two-level TSQR, or when the TSQR's scratch
 * (P leaves x leaf rows x R + 3 P R^2 doubles) exceeds the fixed array
 * (M <= 8192 at R = 32, 29,696 at R = 16, 59,904 at R = 8); CPQR_EHIP if the
 * scratch's device address cannot be obtained or a launch fails.
 */
#define CPQR_QR_NOALLOC_SCRATCH_BYTES (4LL * 1024 * 1024)
cpqr_status cpqr_qr_noalloc(int64_t M, int R, const double *A, double *Q,
                            double *Rout, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* CPQR_H */
