/*
 * mdhp.h - C ABI of the MI355X (gfx950) library that fits exponential-kernel
 * multi-dimensional Hawkes process (MDHP) parameters over many event windows.
 *
 * The method is the MDHP gradient descent solver of "MDHP-Net" (Sec. IV-B):
 * maximise the closed-form log-likelihood of Eq. (5) over (mu, alpha, beta),
 * where Eq. (2) defines the conditional intensity
 *     lambda_m(t) = mu_m + sum_n sum_{k: d_k = n, t_k < t} alpha_mn e^{-beta_mn (t - t_k)}
 * and Eq. (5) (Part1 + Part2 + Part3, derived in Appendix B) is
 *     ll = sum_i log lambda_{d_i}(t_i) - T sum_m mu_m
 *          - sum_{m,n} alpha_mn / beta_mn sum_{k: d_k = n} (1 - e^{-beta_mn (T - t_k)}).
 * The paper's theta is mu here, its D is M and its T_span is T.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Events: one merged, ragged CSR batch.  Window w owns events
 *   [offsets[w], offsets[w+1]); t (FP64) is relative to the window start,
 *   non-decreasing within the window, 0 <= t <= T[w]; dim (int32) is in
 *   [0, M).  Events at equal times never excite each other (the sums of
 *   Eq. (2) and Eq. (5) run over strictly earlier times), so the order
 *   inside a group of equal times does not matter.
 * Parameters (FP32, device memory, row-major):
 *   mu[W][M]; alpha[W][M][M] with alpha[w][m][n] the excitation of target
 *   m by source n (the direction the formula of Eq. (2) gives); beta[W]
 *   (MDHP_BETA_SHARED: one decay per window) or beta[W][M][M]
 *   (MDHP_BETA_PAIR: one decay per pair, the (D, D) beta of Sec. IV-B).
 * Pointers: every array argument is DEVICE memory except mdhp_batch's
 *   n_events/W scalars and the options struct, which are host values.  The
 *   caller owns all buffers; the library allocates only in
 *   mdhp_plan_create and frees in mdhp_plan_destroy; no other call
 *   allocates.
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Compute
 *   calls enqueue work and return; outputs are valid once the stream has
 *   reached them.  A plan must not be used by two streams at once.
 * Errors: every call returns an mdhp_status.  Structural input errors are
 *   found synchronously in mdhp_plan_create.  Compute calls check their
 *   arguments on the host (null pointers, a destroyed plan); they do not
 *   read parameter values on the host, so invalid parameter values (mu <= 0,
 *   alpha < 0, beta <= 0, non-finite) give non-finite results for the
 *   affected windows instead of an error code; mdhp_fit_batch reports them
 *   per window as MDHP_FIT_NONFINITE, or, asked to check its initial values
 *   (mdhp_fit_opts.check_params), returns MDHP_E_PARAM; mdhp_check_params
 *   checks any parameter set.  mdhp_last_error() returns a message for the
 *   last failing call on the calling thread.
 */
#ifndef MDHP_H_
#define MDHP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mdhp_status;
enum {
  MDHP_OK = 0,
  MDHP_E_INVAL = -1,    /* null pointer, M outside [1, 64] ([1, 32] per pair), W < 0, bad option */
  MDHP_E_UNSORTED = -2, /* times decrease inside a window */
  MDHP_E_DOMAIN = -3,   /* t < 0, t > T, dim outside [0, M), T <= 0 or not finite */
  MDHP_E_PARAM = -4,    /* invalid parameter value (checked by the helpers below) */
  MDHP_E_NOMEM = -5,    /* device allocation failed */
  MDHP_E_HIP = -6,      /* a HIP runtime call failed */
  MDHP_E_IO = -7        /* a checkpoint file could not be written or read, or is not one */
};

enum { MDHP_BETA_SHARED = 0, MDHP_BETA_PAIR = 1 };

/* Update rules of mdhp_fit_batch (the paper optimises with an unnamed
 * PyTorch optimizer; these are the rules this library offers; the paper
 * names expectation-maximisation among the estimators of related work).
 * MDHP_OPT_LBFGS is available with one decay per window, MDHP_OPT_EM with
 * fix_beta. */
enum { MDHP_OPT_PGD = 0, MDHP_OPT_PADAM = 1, MDHP_OPT_LBFGS = 2, MDHP_OPT_EM = 3 };

/* Per-window outcome of mdhp_fit_batch.  STALLED: the L-BFGS line search
 * accepted no step (the likelihood no longer increases measurably). */
enum {
  MDHP_FIT_CONVERGED = 0,
  MDHP_FIT_MAX_STEPS = 1,
  MDHP_FIT_NONFINITE = 2,
  MDHP_FIT_STALLED = 3
};

/* Largest L-BFGS memory. */
#define MDHP_MAX_HISTORY 16

/* Largest number of dimensions the kernels support (one decay per window /
 * one decay per pair). */
#define MDHP_MAX_M 64
#define MDHP_MAX_M_PAIR 32

typedef struct mdhp_batch {
  int64_t W;              /* number of windows, >= 0 */
  int64_t n_events;       /* offsets[W] (host value) */
  const int64_t* offsets; /* device int64[W+1], offsets[0] == 0, non-decreasing */
  const double* t;        /* device f64[n_events] */
  const int32_t* dim;     /* device i32[n_events] */
  const double* T;        /* device f64[W], window lengths, > 0 */
} mdhp_batch;

/* Options of mdhp_fit_batch.  All rules work on f = -ll / max(N_w, 1) with
 * the projection Proj: mu >= mu_floor_rel * r_w, alpha >= 0,
 * beta >= beta_floor_rel * r_w, where r_w = max(N_w, 1) / T_w.  Likelihood
 * changes are measured against max(|ll|, N_w, 1): at the optimum the
 * compensator equals N_w (lambda is linear in (mu, alpha)), so N_w is the
 * likelihood's own scale even where ll itself is close to 0.
 *
 * PGD / PADAM: step s = 0, 1, ... evaluates ll_s and its gradient g_s at
 * theta_s; the window stops as converged when s >= 1 and
 * |ll_s - ll_{s-1}| <= ll_tol * max(|ll_s|, N_w, 1), stops as MAX_STEPS when
 * s == max_steps, and otherwise moves to
 *   theta_{s+1} = Proj(theta_s + step(g_s / max(N_w, 1)))
 * with step = lr * g (PGD) or the bias-corrected Adam step (PADAM).
 *
 * LBFGS (projected L-BFGS): per iteration, parameters at their bound whose
 * gradient pushes outward are held fixed; the direction is the two-loop
 * recursion over the last `history` (s, y) pairs applied to the free
 * gradient of f, scaled by s.y / y.y of the newest pair (0.01 / max|g|
 * without history), replaced by that scaled steepest-descent direction if
 * it does not descend; the step is the first of t = 1, 1/2, ... (at most 20
 * trials, each a likelihood + gradient evaluation) whose projected point
 * satisfies f(x') <= f(x) + 1e-4 g.(x' - x); a pair enters the history if
 * s.y > 1e-10 |s| |y|.  The window stops as converged when an accepted step
 * changes ll by at most ll_tol * max(|ll|, N_w, 1) or the free gradient is zero,
 * as MAX_STEPS after max_steps accepted steps, and as STALLED when no trial
 * is accepted.  lr, adam_* are not used.
 *
 * EM (expectation-maximisation on the branching structure: every event is
 * either a background event of its dimension or the offspring of one
 * earlier event): the decays stay at their initial values (fix_beta must be
 * set).  Step s evaluates ll_s, stops as PGD does, and otherwise sets
 *   mu_m    <- max(mu_m * G_m / T_w, mu_floor_rel * r_w),
 *   alpha_mn <- alpha_mn * G_mn / C_mn   (unchanged where C_mn = 0),
 * where G_m = sum_{i: d_i = m} 1 / lambda_i (mu_m G_m is the expected number
 * of background events of dimension m), G_mn = sum_{i: d_i = m} R_mn(i) /
 * lambda_i (alpha_mn G_mn: the expected number of dimension-m events
 * triggered by dimension-n events) and C_mn = sum_{k: d_k = n}
 * (1 - e^{-beta_mn (T_w - t_k)}) / beta_mn (Part3's coefficient, the
 * exposure).  Each step does not decrease ll; the optimum over (mu, alpha)
 * at fixed decays is its fixed point (there G_m = T_w and G_mn = C_mn
 * wherever the bound is not active).  lr, history and adam_* are not used.
 *
 * check_params: non-zero makes mdhp_fit_batch validate the initial values
 * first (mu > 0, alpha >= 0, beta > 0, all finite: the domain of Eq. (2)
 * and Eq. (5)) and return MDHP_E_PARAM without fitting if any window
 * violates them; the call then waits for the check on `stream` (so it must
 * not be captured into a graph).  Zero (the default) keeps the call
 * asynchronous: initial values are not read on the host, the first update
 * projects them onto the feasible set, and a window whose evaluation is not
 * finite ends as MDHP_FIT_NONFINITE. */
typedef struct mdhp_fit_opts {
  int32_t max_steps; /* >= 0 */
  int32_t optimizer; /* MDHP_OPT_PGD, MDHP_OPT_PADAM, MDHP_OPT_LBFGS or MDHP_OPT_EM */
  int32_t fix_beta;  /* non-zero: beta is not updated */
  int32_t history;   /* L-BFGS memory, 0 (= 8) .. MDHP_MAX_HISTORY */
  double lr;         /* > 0 (PGD, PADAM) */
  double ll_tol;     /* >= 0 */
  double mu_floor_rel;
  double beta_floor_rel;
  double adam_b1, adam_b2, adam_eps;
  int32_t check_params; /* non-zero: validate the initial values (synchronous) */
  int32_t reserved;     /* 0 */
} mdhp_fit_opts;

typedef struct mdhp_plan mdhp_plan;

/* Validates a batch and prepares it for the kernels (Sec. IV-B "Stage 1:
 * Initialization" is the paper's counterpart).  Synchronous: runs the
 * preparation kernel on `stream`, waits for it and returns
 * MDHP_E_UNSORTED / MDHP_E_DOMAIN for bad events.  On success *out owns a
 * compact copy of the events (FP32 gaps and FP32 distances T - t to the
 * window's end, both computed in FP64, u8 dims: 9 B per event; per-pair
 * plans add the FP32 gap to the previous event of the same dimension: 13 B),
 * the window order (largest first) and the workspace.  M in [1, 64] with
 * MDHP_BETA_SHARED, [1, 32] with MDHP_BETA_PAIR. */
mdhp_status mdhp_plan_create(const mdhp_batch* batch, int32_t M, int32_t beta_mode, void* stream,
                             mdhp_plan** out);

/* Frees a plan (NULL is accepted).  Waits for the device to finish with it. */
void mdhp_plan_destroy(mdhp_plan* plan);

/* Number of windows / events / dimensions of a plan (0 for NULL). */
int64_t mdhp_plan_windows(const mdhp_plan* plan);
int64_t mdhp_plan_events(const mdhp_plan* plan);
int32_t mdhp_plan_dims(const mdhp_plan* plan);

/* Log-likelihood of Eq. (5) per window: ll[W] (device f64).  Part1 is
 * evaluated by a segmented scan of the exponential-kernel recursion, Part2
 * and Part3 in closed form (Appendix B) from the scan's end state, or, for a
 * decay that is slow against the window (small beta T), from the events'
 * distances to T, where the end-state form would cancel; per-window sums are
 * reduced in FP64. */
mdhp_status mdhp_loglik(mdhp_plan* plan, const float* mu, const float* alpha, const float* beta,
                        double* ll, void* stream);

/* Log-likelihood and its gradient (the ascent direction d ll / d theta, in
 * the parameters' layouts): g_mu[W][M], g_alpha[W][M][M], g_beta[W] or
 * [W][M][M] (device f32); ll[W] (device f64).  One pass per window; no
 * backward scan. */
mdhp_status mdhp_grad(mdhp_plan* plan, const float* mu, const float* alpha, const float* beta,
                      double* ll, float* g_mu, float* g_alpha, float* g_beta, void* stream);

/* Fit of every window in one persistent launch (windows largest first from
 * an atomic queue; the whole iteration loop of a window runs inside one
 * workgroup).  mu/alpha/beta hold the initial values on entry and the
 * fitted values on return; ll[W] is ll at the returned parameters,
 * steps[W] the number of updates applied, status[W] one of MDHP_FIT_*,
 * and evals[W] (optional, may be NULL) the number of likelihood + gradient
 * evaluations.  A window whose evaluation is not finite returns the
 * parameters of that evaluation with status MDHP_FIT_NONFINITE. */
mdhp_status mdhp_fit_batch(mdhp_plan* plan, const mdhp_fit_opts* opts, float* mu, float* alpha,
                           float* beta, double* ll, int32_t* steps, int32_t* status,
                           int32_t* evals, void* stream);

/* Cold start of every window (the initial point of the fits and the warm
 * start's fallback; the paper leaves the initial point of its solver open,
 * so this is a stated choice): mu_m = 0.5 max(N_m, 0.5) / T_w (half the
 * window's rate of dimension m, N_m its events), beta = 1 (every entry in
 * per-pair mode) and alpha_mn = 0.5 / M, a branching matrix of spectral
 * radius 0.5.  mu [W][M], alpha [W][M][M], beta [W] or [W][M][M] are device
 * memory owned by the caller.  Enqueued on stream. */
mdhp_status mdhp_cold_start(mdhp_plan* plan, float* mu, float* alpha, float* beta, void* stream);

/* Allocation-free likelihood and gradient, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation.  No plan: the batch (device pointers, as for
 * mdhp_plan_create, one decay per window: mu [W][M], alpha [W][M][M],
 * beta [W]) is prepared and evaluated on `stream` in one asynchronous call,
 * with the same Eq. (5) likelihood and gradient as mdhp_grad (lane-per-
 * dimension kernels for every M in [1, 64], windows in their given order).
 * The call allocates nothing: the prepared events live in one fixed device
 * array of the library (MDHP_STATIC_BYTES, each GPU it runs on holds its
 * own copy until the process ends), whose address is looked up once per
 * device on its first call there.  Every call on a GPU shares that array:
 * calls that overlap on one GPU (other streams, other host threads) race
 * and must be serialised by the caller.  Limits: W <= MDHP_STATIC_MAX_WINDOWS
 * and n_events <= MDHP_STATIC_MAX_EVENTS (MDHP_E_INVAL beyond).  g_mu,
 * g_alpha, g_beta: all three (gradient of ll) or all NULL (likelihood only).
 * The host reads nothing back, so events are validated on the device: a
 * window whose events are unsorted or out of range, or whose offsets are
 * inconsistent, gets ll = NaN (and NaN gradients); offsets are clamped to
 * [0, n_events] before any event is read. */
#define MDHP_STATIC_MAX_EVENTS 4194304
#define MDHP_STATIC_MAX_WINDOWS 65536
#define MDHP_STATIC_BYTES 56623616
mdhp_status mdhp_grad_static(const mdhp_batch* batch, int32_t M, const float* mu,
                             const float* alpha, const float* beta, double* ll, float* g_mu,
                             float* g_alpha, float* g_beta, void* stream);

/* Checks parameter values on the device (mu > 0, alpha >= 0, beta > 0, all
 * finite) and returns MDHP_E_PARAM if any window violates them.
 * Synchronous on `stream`. */
mdhp_status mdhp_check_params(mdhp_plan* plan, const float* mu, const float* alpha,
                              const float* beta, void* stream);

/* ------------------------------------------------------------------------
 * Schedule autotuning.  A plan runs with one of a few schedules, chosen per
 * plan because the best one depends on its window sizes:
 *   kind 1 (one decay per window, M <= 16): the number of events from which
 *     a window is run by a whole workgroup of 256 lanes instead of one
 *     wavefront of 64 (512, 1024, 2048, 4096 or MDHP_TEAM_NEVER; the events'
 *     layout in the plan depends on it; default 1024);
 *   kind 2 (one decay per window, 16 < M <= 64): the events per
 *     reduce-scatter of the intensity sums (4, 8 or 16 for M > 32; 4 or 8
 *     for M <= 32; default 8), or for M > 32 MDHP_SCATTER_MFMA: the
 *     alpha contraction of Eq. (2) for blocks of 16 events as one product
 *     R (16 x 64) alpha^T (64 x 64) on the matrix cores (FP32 MFMA), of
 *     which each event keeps its own target's entry;
 *   kind 0 (per-pair decays): nothing to choose.
 * The schedule changes the order of floating-point sums, never the result
 * beyond rounding. */
#define MDHP_TUNE_MAX 8
#define MDHP_TEAM_NEVER 2147483647
#define MDHP_SCATTER_MFMA 1

typedef struct mdhp_tune_result {
  int32_t kind;                 /* 0, 1 or 2 as above */
  int32_t n;                    /* candidates timed */
  int32_t chosen;               /* index of the kept candidate */
  int32_t value[MDHP_TUNE_MAX]; /* candidate schedules */
  float ms[MDHP_TUNE_MAX];      /* milliseconds of the fastest timed repetition */
} mdhp_tune_result;

/* Times every candidate schedule of the plan on its own windows from the
 * cold start (mdhp_cold_start) and keeps the fastest.  opts == NULL times
 * `reps` evaluations of mdhp_grad; otherwise `reps` calls of mdhp_fit_batch
 * with opts (each after one untimed warm-up).  `batch` must be the batch the
 * plan was created from (kind 1 re-prepares it per candidate; unused for
 * kinds 0 and 2, may be NULL there).  Synchronous on `stream`; allocates and
 * frees device scratch memory (parameter and output copies), so it must not
 * be called during stream capture.  On error the plan keeps a valid
 * schedule.  Results in *result. */
mdhp_status mdhp_plan_autotune(mdhp_plan* plan, const mdhp_batch* batch, const mdhp_fit_opts* opts,
                               int32_t reps, mdhp_tune_result* result, void* stream);

/* Sets the plan's schedule to `value` (a candidate of its kind, else
 * MDHP_E_INVAL) without timing; `batch` as for mdhp_plan_autotune.
 * Synchronous on `stream` when the events are re-prepared. */
mdhp_status mdhp_plan_set_schedule(mdhp_plan* plan, const mdhp_batch* batch, int32_t value,
                                   void* stream);

/* The plan's current schedule value (0 for kind 0 or a NULL plan). */
int32_t mdhp_plan_schedule(const mdhp_plan* plan);

/* Events per window and dimension as the plan counted them at creation
 * (the N_m of the cold start, Sec. IV-B): counts [W][M] int32, device
 * memory, caller-owned, in the batch's window order.  Enqueued on stream
 * (a device-to-device copy); MDHP_E_INVAL for an invalid plan or a null
 * pointer with W > 0. */
mdhp_status mdhp_plan_dim_counts(const mdhp_plan* plan, int32_t* counts, void* stream);

/* mdhp_plan_create with a schedule chosen beforehand (a candidate of the
 * plan's kind, e.g. from an earlier mdhp_plan_autotune of the same batch
 * shape; 0 = default), prepared once in that layout.  MDHP_E_INVAL for a
 * value that is not a candidate. */
mdhp_status mdhp_plan_create_scheduled(const mdhp_batch* batch, int32_t M, int32_t beta_mode,
                                       int32_t schedule, void* stream, mdhp_plan** out);

/* ------------------------------------------------------------------------
 * Learned warm start (an addition around the paper's solver, which fits
 * every window from scratch): count-histogram features, a 3-layer ReLU MLP
 * trained on the GPU with BF16 MFMA GEMMs (FP32 accumulation and master
 * weights, Adam), and the epilogue that turns its prediction into initial
 * parameters with the cold start as fallback.
 * ------------------------------------------------------------------------ */

/* Features of every window of a batch (device pointers as in mdhp_batch):
 * x[w][m * bins + b] = log1p(count_{m,b} * bins / T_w) as BF16 (uint16 bit
 * patterns), where event (t, m) falls in bin floor(t * bins / T_w) (FP64,
 * clamped to bins - 1).  x is device memory [W][M * bins]; M * bins <= 16384. */
mdhp_status mdhp_features(const mdhp_batch* batch, int32_t M, int32_t bins, uint16_t* x,
                          void* stream);

typedef struct mdhp_surrogate mdhp_surrogate;

/* MLP in_dim -> hidden -> hidden -> out_dim with ReLU after the two hidden
 * layers; He-uniform weights from SplitMix64(seed), zero biases.  Allocates
 * weights, Adam state and activations for batches of up to max_batch rows.
 * Synchronous.  Parameters are one FP32 buffer: W1[hidden][in], b1[hidden],
 * W2[hidden][hidden], b2[hidden], W3[out][hidden], b3[out]. */
mdhp_status mdhp_surrogate_create(int32_t in_dim, int32_t hidden, int32_t out_dim,
                                  int32_t max_batch, uint64_t seed, mdhp_surrogate** out);
void mdhp_surrogate_destroy(mdhp_surrogate* s);

/* Number of FP32 parameters; copies of them to / from a caller buffer
 * (device memory, n_params floats).  set_weights also refreshes the BF16
 * copies the GEMMs read.  Enqueued on stream. */
int64_t mdhp_surrogate_num_params(const mdhp_surrogate* s);
mdhp_status mdhp_surrogate_get_weights(mdhp_surrogate* s, float* dst, void* stream);
mdhp_status mdhp_surrogate_set_weights(mdhp_surrogate* s, const float* src, void* stream);

/* y[B][out_dim] (device f32) = MLP(x[B][in_dim] BF16).  B <= max_batch. */
mdhp_status mdhp_surrogate_forward(mdhp_surrogate* s, const uint16_t* x, int32_t B, float* y,
                                   void* stream);

/* Copies the last forward pass's BF16 hidden activations (first B rows of
 * each hidden layer, [B][hidden]) to caller device buffers. */
mdhp_status mdhp_surrogate_get_hidden(mdhp_surrogate* s, int32_t B, uint16_t* h1, uint16_t* h2,
                                      void* stream);

/* Forward pass, mean squared error against target[B][out_dim] (device f32)
 * into *loss (device f64), and the gradient of that loss with respect to
 * every parameter (same layout as the weights), kept inside the surrogate;
 * get_gradients copies them to a caller device buffer. */
mdhp_status mdhp_surrogate_backward(mdhp_surrogate* s, const uint16_t* x, int32_t B,
                                    const float* target, double* loss, void* stream);
mdhp_status mdhp_surrogate_get_gradients(mdhp_surrogate* s, float* dst, void* stream);

/* One Adam step (bias-corrected) on the master weights with the last
 * backward pass's gradients; refreshes the BF16 copies. */
mdhp_status mdhp_surrogate_adam(mdhp_surrogate* s, float lr, float b1, float b2, float eps,
                                void* stream);

/* backward followed by adam(lr, 0.9, 0.999, 1e-8). */
mdhp_status mdhp_surrogate_train_step(mdhp_surrogate* s, const uint16_t* x, int32_t B,
                                      const float* target, float lr, double* loss,
                                      void* stream);

/* Checkpoint of a surrogate, for resuming training or serving a trained
 * network (the library's addition; the paper has no learned warm start).
 * File layout (host byte order, little-endian on every supported host):
 *   char magic[8] = "MDHPSUR1"; int32 version = 1; int32 in_dim, hidden,
 *   out_dim; int64 n_params; int64 adam_step; int64 n_extra;
 *   float32 weights[n_params]; float32 adam_m1[n_params];
 *   float32 adam_m2[n_params]; float32 extra[n_extra].
 * `extra` (host memory, may be NULL when n_extra is 0) is caller data kept
 * with the network, e.g. the normalisation of its targets.
 * save: waits for `stream`, copies the FP32 master weights and both Adam
 * moments to the host and writes them with the step count; MDHP_E_IO if the
 * file cannot be written.
 * load: reads such a file into a surrogate of the same in_dim, hidden and
 * out_dim (else MDHP_E_INVAL), restores weights, moments and step, refreshes
 * the BF16 copy and waits for `stream`; MDHP_E_IO for a missing, truncated
 * or foreign file.  *n_extra receives the stored extra count; at most
 * extra_cap values are copied to extra (NULL: none). */
mdhp_status mdhp_surrogate_save(mdhp_surrogate* s, const char* path, const float* extra,
                                int64_t n_extra, void* stream);
mdhp_status mdhp_surrogate_load(mdhp_surrogate* s, const char* path, float* extra,
                                int64_t extra_cap, int64_t* n_extra, void* stream);

/* Warm start for a plan with one decay per window.  pred[W][M + M*M + 1]
 * (device f32) is the network output for the plan's windows, z-scored:
 * y = pred * stdv + mean gives, in the parameter layout order,
 * log(mu_m T / max(N_m, 0.5)) (the log of mu_m over the window's rate of
 * dimension m), the branching entries alpha_mn / beta, and log beta.
 * Writes beta = exp(y_beta), mu_m = exp(y_m) max(N_m, 0.5) / T (both
 * clamped to opts' floors) and alpha_mn = max(y_mn, 0) beta, evaluates ll
 * at them and at the cold start
 * (mu_cold, alpha_cold, beta_cold), keeps the cold start for windows where
 * it is at least as likely or the warm one is not finite, and records the
 * choice in used_warm[W] (1 = warm).  Enqueued on stream. */
mdhp_status mdhp_warm_start(mdhp_plan* plan, const float* pred, const float* mean,
                            const float* stdv, const mdhp_fit_opts* opts, const float* mu_cold,
                            const float* alpha_cold, const float* beta_cold, float* mu,
                            float* alpha, float* beta, int32_t* used_warm, void* stream);

/* ------------------------------------------------------------------------
 * Simulation of MDHP windows on the device: Ogata's thinning for the model of
 * Eq. (2) with one decay per window (M <= 64) or per pair
 * (M <= MDHP_SIM_PAIR_MAX_M), one window per wavefront, FP64 throughout.
 * The total intensity at the current time bounds it until the next event;
 * a candidate s' = s + Exp(bound) is accepted with probability
 * sum_m lambda_m(s') / bound and takes the first dimension whose cumulative
 * intensity reaches a uniform fraction of the total.  Window w draws the
 * SplitMix64 stream (seed, first_window + w) (Steele, Lea and Flood 2014;
 * one word from a generator seeded with seed ^ 0x6A09E667F3BCC909, keyed with
 * the window index), so a window does not depend on the batch it is
 * simulated in.
 *
 * mode MDHP_SIM_UNTIL_T: window w runs on [0, T_in[w]] with room for
 *   offsets[w+1] - offsets[w] events; n_out[w] = its events, T_out[w] =
 *   T_in[w]; a window with more events than its room stops there with
 *   n_out[w] = -1.
 * mode MDHP_SIM_COUNT: window w gets exactly offsets[w+1] - offsets[w]
 *   events (n_out[w]) and ends at the time of the next accepted one
 *   (T_out[w]); T_in is not read.
 * In either mode n_out[w] = -2 where the window cannot be drawn: a total
 * intensity that is negative, infinite or NaN at some step, a zero one
 * while MDHP_SIM_COUNT still owes events, or T_in[w] negative or not
 * finite; the window's outputs are then undefined.
 * Device memory, caller-owned: mu [W][M], alpha [W][M][M] (alpha[w][m][n]:
 * source n excites target m), beta [W] or [W][M][M], T_in [W], offsets
 * [W+1]; outputs t_out [offsets[W]] (event times), dim_out [offsets[W]],
 * written from offsets[w] on, n_out [W], T_out [W].  Parameters are not
 * validated beyond that check (mu > 0, alpha >= 0, beta > 0 and a stable
 * branching matrix are the caller's; an unstable one fills the room).
 * MDHP_E_INVAL for bad sizes or modes.  Enqueued on stream. */
#define MDHP_SIM_UNTIL_T 0
#define MDHP_SIM_COUNT 1
#define MDHP_SIM_PAIR_MAX_M 32
mdhp_status mdhp_simulate(int64_t W, int32_t M, int32_t beta_mode, const double* mu,
                          const double* alpha, const double* beta, int32_t mode,
                          const double* T_in, const int64_t* offsets, uint64_t seed,
                          int64_t first_window, double* t_out, int32_t* dim_out, int64_t* n_out,
                          double* T_out, void* stream);

/* Injection times of the paper's time-exciting attack strategies (attack
 * rates g(t) of Sec. III's strategy table) drawn by its three samplers
 * (appendix, sampling algorithms), one attack window per GPU thread:
 *   MDHP_ATTACK_PLA  g = a t^b                                  params (a, b)
 *   MDHP_ATTACK_DEA  g = W1 a1 t^(a1 - 1) for t < t1, W2 a2 e^(c (t - t1)) after
 *                                                  params (W1, a1, W2, a2, c, t1)
 *   MDHP_ATTACK_ASA  g = C e^(c t) / (1 + e^(c (t - t0)))^2     params (C, c, t0)
 *   MDHP_ATTACK_DAM  g = w a1 t^(a1 - 1) + (1 - w) a2 e^(a2 t)  params (w, a1, a2)
 *   MDHP_SAMPLER_NPP candidates with Exp gaps of mean 1 / r, a candidate t
 *     kept when a Uniform(0, g_max) draw is below g(t);
 *   MDHP_SAMPLER_ND  candidates with gaps |Normal(1 / r, 1 / (2 r))|, kept
 *     with probability g(t) / g_max;
 *   MDHP_SAMPLER_DRP DAM (a1 = params[1], a2 = params[2]) whose weight w is
 *     drawn per third of the range from U(0, 1/3), U(1/3, 2/3), U(2/3, 1),
 *     then NPP's thinning (strategy[a] is not read).
 * r = params[7] (512 when 0); g_max is the largest g on a grid of 4,097
 * points of the range (the paper takes it from evaluations of g).  Attack a
 * draws SplitMix64 stream (seed, first + a) as mdhp_simulate does.  Device
 * memory, caller-owned: strategy [A], sampler [A], params [A][8], range
 * [A][2] (t_min, t_max; the paper normalises windows to [0, 1]), offsets
 * [A+1] (room per attack); outputs t_out (increasing times from offsets[a]
 * on) and n_out [A]: -1 where the room was too small, -2 where the range
 * is not one (t_max < t_min, NaN or infinite ends) or
 * r (t_max - t_min) exceeds 2^24 candidates.  MDHP_E_INVAL for bad sizes;
 * the rate parameters are the caller's.  Enqueued on stream. */
#define MDHP_ATTACK_PLA 0
#define MDHP_ATTACK_DEA 1
#define MDHP_ATTACK_ASA 2
#define MDHP_ATTACK_DAM 3
#define MDHP_SAMPLER_NPP 0
#define MDHP_SAMPLER_ND 1
#define MDHP_SAMPLER_DRP 2
mdhp_status mdhp_attack_times(int64_t A, const int32_t* strategy, const int32_t* sampler,
                              const double* params, const double* range, const int64_t* offsets,
                              uint64_t seed, int64_t first, double* t_out, int64_t* n_out,
                              void* stream);

/* ------------------------------------------------------------------------
 * The MDHP-LSTM layer (Sec. IV, "MDHP-LSTM", Eq. (7)), FP32, forward and
 * backward.  For B sequences of L inputs x_t (width D), hidden width H and
 * each sequence's fitted window parameters (alpha, beta, theta = mu) and
 * length T_span:
 *   hks = tanh(A vec(alpha) - B (beta T_span) + C theta)      once per sequence
 *   z_t = W x_t + U h_{t-1} + b;  i, f, o = sigmoid, g = tanh of its blocks
 *   c_t = hks * (f c_{t-1} + i g);  h_t = o tanh(c_t);  h_{-1} = c_{-1} = 0.
 * hks carries only window quantities, so it is computed once and gates
 * every step; the paper's readout y = W_y h is a plain linear layer left to
 * the caller.  Gate blocks are ordered i, f, g, o (torch.nn.LSTM's order).
 * Layouts (row-major, device memory, caller-owned): x [B][L][D], W [4H][D],
 * U [4H][H], bias [4H], Whks [H][Kf] = [A | B | C] with Kf = M^2 + Kb + M
 * (Kb = 1 for one decay per window, M^2 for one per pair), alpha [B][M][M],
 * beta [B] or [B][M][M], T_span [B], theta [B][M]; h [B][L][H] out.
 * `saved` (mdhp_lstm_sizes' first count of floats) receives what the
 * backward pass reads: gate activations [B][L][4H], cells [B][L][H], hks
 * [B][H] and the features [B][Kf]; `work` (its second count) is scratch.
 * H must be 64, 128 or 256; MDHP_E_INVAL for bad sizes or null pointers.
 * Enqueued on stream. */
typedef struct mdhp_lstm_dims {
  int32_t B;         /* sequences */
  int32_t L;         /* steps per sequence, >= 1 */
  int32_t D;         /* input width, >= 1 */
  int32_t H;         /* hidden width: 64, 128 or 256 */
  int32_t M;         /* MDHP dimensions, 1..64 */
  int32_t beta_mode; /* MDHP_BETA_SHARED or MDHP_BETA_PAIR */
} mdhp_lstm_dims;

/* Floats of the saved state and of the workspace for these dimensions. */
mdhp_status mdhp_lstm_sizes(const mdhp_lstm_dims* dims, int64_t* saved_floats,
                            int64_t* work_floats);
mdhp_status mdhp_lstm_forward(const mdhp_lstm_dims* dims, const float* x, const float* W,
                              const float* U, const float* bias, const float* Whks,
                              const float* alpha, const float* beta, const float* T_span,
                              const float* theta, float* h, float* saved, float* work,
                              void* stream);
/* Gradients of a loss whose gradient with respect to every output h_t is
 * dh [B][L][H]: dx [B][L][D], dW [4H][D], dU [4H][H], dbias [4H], dWhks
 * [H][Kf] (= [dA | dB | dC]) and dfeat [B][Kf] (with respect to vec(alpha),
 * beta T_span and theta).  x, W, U, Whks and h are the forward pass's;
 * `saved` is the forward pass's and is consumed (its gate activations are
 * overwritten by the gradients of their pre-activations).  Outputs are
 * overwritten, not accumulated.  With B = 0 the arrays of B rows may be
 * null and the weight gradients come out zero. */
mdhp_status mdhp_lstm_backward(const mdhp_lstm_dims* dims, const float* x, const float* W,
                               const float* U, const float* Whks, const float* h, float* saved,
                               const float* dh, float* dx, float* dW, float* dU, float* dbias,
                               float* dWhks, float* dfeat, float* work, void* stream);

/* Phase timing of the MDHP-LSTM passes, for profiling.  With enable = 1 the
 * following calls of mdhp_lstm_forward and mdhp_lstm_backward record HIP
 * events (created on the device current at the first enable) between their
 * phases, on their stream; mdhp_lstm_phase_ms waits for the last call of
 * each pass and writes its phase durations in ms (-1 for a pass not run
 * since timing was enabled; either pointer may be null):
 *   forward  [MDHP_LSTM_FWD_PHASES]: features and packing of U, the hks
 *            GEMM, the input GEMM (for D <= 256, where the recurrence forms
 *            the input products itself: the packing of W), the recurrence;
 *   backward [MDHP_LSTM_BWD_PHASES]: packing of U, the recurrence (with
 *            the bias gradient), the dx, dW and dU GEMMs, the Hawkes-gate
 *            gradients.
 * Process-wide state: one timing caller at a time. */
#define MDHP_LSTM_FWD_PHASES 4
#define MDHP_LSTM_BWD_PHASES 6
mdhp_status mdhp_lstm_timing(int32_t enable);
mdhp_status mdhp_lstm_phase_ms(float* fwd_ms, float* bwd_ms);

/* Static description of a status code. */
const char* mdhp_status_string(mdhp_status status);

/* Copies the calling thread's last error message into buf (NUL-terminated,
 * truncated to n bytes) and returns the last error's status. */
mdhp_status mdhp_last_error(char* buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* MDHP_H_ */
