/*
 * libotlm -- batched entropic Optimal Transport Linear Model solver for AMD
 * Instinct MI355X (gfx950).
 *
 * The library solves, for many target spectra y_b at once, the regularised
 * OTLM problem of Kacprzak et al., "Scalable Approximate Algorithms for
 * Optimal Transport Linear Models" (eq. OTLM, in the scaling-algorithm form
 * of section "Scaling Algorithm Framework for OTLM"):
 *
 *   min_{Q >= 0, w >= 0}  eps KL(Q || K) + lambda L(Q^T 1 | y) + alpha R(w)
 *   subject to Q 1 = D w,           K = exp(-C / eps),
 *
 * with the scaling iteration of Algorithm 1: per iteration
 *   s = K v;  w <- wMMstep(s, Z | D)  (Table 2 / Appendix A);  u = D w / s;
 *   t = K^T u;  p = prox_L(t | y)      (Table 1);              v = p / t.
 * The plan is Q = diag(u) K diag(v) (row i = source bin, column j = target).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers to contiguous row-major arrays,
 *    owned by the caller; the library never frees them.  Batched arrays are
 *    [B, n] (one spectrum per row) or [B, k].
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it; a call returns once its work is enqueued, except
 *    where a comment says it synchronises.
 *  - Return value: OTLM_OK (0) or a negative otlm_status.  On a negative
 *    return nothing has been written to the outputs unless stated.  Argument
 *    errors are detected before any launch.
 *  - Not thread-safe per kernel object: calls that share an otlm_kernel must
 *    be serialised by the caller (they share its workspace).
 */
#ifndef OTLM_H
#define OTLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct otlm_kernel_s* otlm_kernel;

typedef enum {
  OTLM_OK = 0,
  OTLM_E_INVALID = -1,      /* bad argument (null pointer, size, parameter range) */
  OTLM_E_HIP = -2,          /* a HIP runtime call failed                        */
  OTLM_E_NOMEM = -3,        /* device allocation failed                         */
  OTLM_E_UNSUPPORTED = -4   /* valid request this build does not implement      */
} otlm_status;

/* Target datafit L (Table 1).  L2_TV is lambda * L2 + lambda2 * TV with
 * prox_{L2} o prox_{TV}; POISSON is the negative Poisson log-likelihood with
 * the reciprocal reading 1 / W_0 of the table's last row. */
typedef enum {
  OTLM_FIT_BALANCED = 0, OTLM_FIT_KL = 1, OTLM_FIT_TV = 2, OTLM_FIT_L2 = 3,
  OTLM_FIT_L2_TV = 4, OTLM_FIT_POISSON = 5
} otlm_datafit;

/* Weight penalty alpha R(w) (Table 2, Appendix A): none; alpha ||w||_1;
 * (alpha/2) ||w||_2^2; alpha ||w||_1 + (beta/2) ||w||_2^2. */
typedef enum {
  OTLM_PEN_NONE = 0, OTLM_PEN_L1 = 1, OTLM_PEN_L2SQ = 2, OTLM_PEN_ELASTIC = 3
} otlm_penalty;

typedef enum {
  OTLM_PREC_FP32 = 0,          /* FP32 kernel products on MFMA, FP32 state             */
  OTLM_PREC_BF16 = 1           /* BF16 kernel products (FP32 accumulate), FP32 state   */
} otlm_precision;

typedef enum {
  OTLM_REFINE_NONE = 0,        /* no refinement phase                                   */
  OTLM_REFINE_FP32 = 1,        /* FP32 products and state                               */
  OTLM_REFINE_FP64 = 2         /* FP64 products (MFMA f64) and state                    */
} otlm_refine;

enum { OTLM_WSTEP_MM = 0, OTLM_WSTEP_EXACT = 1 };

/* Per-spectrum outcome flags written to status[b]. */
enum {
  OTLM_S_CONVERGED = 1,   /* the stopping test passed                                */
  OTLM_S_MAX_ITER = 2,    /* stopped at the iteration cap                            */
  OTLM_S_NONFINITE = 4,   /* a NaN/Inf appeared; the spectrum was frozen             */
  OTLM_S_STAGNATED = 8,   /* the weight change stopped improving for 6 tests: the
                             noise floor of the phase precision was reached        */
  OTLM_S_FALLBACK = 16,   /* (with another flag) the warm start failed the probe
                             and the spectrum was solved from the cold start       */
  OTLM_S_ABSORBED = 32    /* (with another flag) the scalings of the FP32 bulk
                             phase exceeded exp(+-absorb_tau); the spectrum left
                             the bulk phase early and was solved in the FP64
                             state                                                */
};

/* Solver parameters.  A solve has a bulk phase in precision `prec` and, when
 * `refine` is not NONE, a refinement phase in precision `refine` that starts
 * from the bulk result.  Each phase freezes a spectrum once its own test
 * passes: the stopping rule of "while not converged" is
 *   sum|u o (K v) - D w| / sum(D w) <= tol_phase   and
 *   d rho / (1 - rho) <= tol_phase, with d = max|w - w'| / max|w| the weight
 *   change since the previous test (w' = weights then) and rho = d / d_prev
 *   its observed contraction, or d below the phase precision's resolution and
 *   no longer shrinking.
 * tol_phase is `bulk_tol` for a bulk phase followed by refinement, `tol`
 * otherwise. */
typedef struct {
  double eps;            /* entropic regulariser, > 0 (must equal the kernel's)   */
  double lambda;         /* datafit weight, >= 0                                   */
  double lambda2;        /* TV weight of OTLM_FIT_L2_TV, >= 0                      */
  double alpha;          /* penalty weight, >= 0 (> 0 for L2SQ)                    */
  double beta;           /* quadratic weight of OTLM_PEN_ELASTIC, > 0 there        */
  double tol;            /* final stopping tolerance, >= 0 (0 = run to the caps)   */
  double bulk_tol;       /* bulk-phase tolerance when a refinement follows, >= 0   */
  double warm_probe;     /* > 0 with warm = 1: at the first convergence test, a
                            spectrum whose weight change over the interval
                            exceeds warm_probe relative to the weights in the l1
                            norm, sum|w - w_start| / sum|w| (or is not finite),
                            restarts from the cold start and is flagged
                            OTLM_S_FALLBACK; 0: no probe                          */
  double absorb_tau;     /* with REFINE_FP64: at every convergence test of the
                            bulk phase a spectrum with |log u_i| or |log v_i| >
                            absorb_tau moves to the FP64 phase (whose state spans
                            exp(+-709)) and is flagged OTLM_S_ABSORBED; 0: off;
                            default 30                                            */
  int32_t max_iter;      /* iteration cap of the bulk phase, >= 1                  */
  int32_t check_every;   /* convergence test cadence in iterations, >= 1           */
  int32_t fit;           /* otlm_datafit                                           */
  int32_t pen;           /* otlm_penalty                                           */
  int32_t prec;          /* otlm_precision of the bulk phase                       */
  int32_t refine;        /* otlm_refine                                            */
  int32_t refine_sweeps; /* iteration cap of the refinement phase, >= 1 if used    */
  int32_t warm;          /* 0: cold start (w0_j = sum(y)/(k x_j), v = 1);
                            1: start from the W and logV arrays passed in          */
  int32_t wstep;         /* weight step per iteration: OTLM_WSTEP_MM (one MM step,
                            Table 2, as in Algorithm 1) or OTLM_WSTEP_EXACT (the
                            weight prox ProxP solved by an active-set Newton
                            method, the run-to-convergence alternative of
                            subsection "Iterative Algorithm for OTLM"; needs
                            kdim <= 64 and n <= 1024; the first 3 iterations of
                            a cold start take the MM step)                          */
  int32_t inner_max;     /* Newton iterations per weight prox (WSTEP_EXACT), >= 1  */
  int32_t refine_check_every; /* convergence test cadence of the refinement phase,
                            >= 0 (0: check_every); the refinement phase is short
                            and its stopping rule needs two test intervals, so a
                            short cadence ends it sooner; default 2              */
} otlm_params;

/* Fill `p` with defaults: KL datafit, no penalty, eps = lambda = 1, tol 1e-6,
 * bulk_tol 1e-4, absorb_tau 30, no warm probe, max_iter 1000, check_every 10, FP32, no refinement
 * (refine_sweeps 200 and refine_check_every 2 when enabled), cold start, one MM
 * step per iteration, inner_max 5. */
void otlm_default_params(otlm_params* p);

/* Build the Gibbs kernel K = exp(-C / eps) (Algorithm 1, initialisation).
 *   C       device, FP64, [n, n] row-major cost (row = source bin i, column =
 *           target bin j); read only during the call.  The OTLM problem has
 *           the same bins on both sides, so C is square.
 *   n       number of bins, 1 <= n <= 16384.
 *   eps     > 0.
 *   out     receives an opaque handle owning device copies of K (FP32 and
 *           BF16), K^T when C is not symmetric, and sum(K) in FP64.
 * Synchronises `stream` (it checks C for symmetry on the host).
 * Errors: OTLM_E_INVALID (null, n out of range, eps <= 0), OTLM_E_NOMEM,
 * OTLM_E_HIP. */
int otlm_make_kernel(const double* C, int64_t n, double eps, void* stream, otlm_kernel* out);

/* Release a kernel object and every workspace it cached.  NULL is a no-op.
 * Synchronises the device. */
int otlm_free_kernel(otlm_kernel k);

/* Number of bins and symmetry flag of a kernel object. */
int otlm_kernel_info(otlm_kernel k, int64_t* n, int32_t* symmetric, double* eps);

/* Run Algorithm 1 on B target spectra that share K and the dictionary D.
 *   D       device FP32 [n, kdim], non-negative, every column sum > 0 (the
 *           paper's X; column sums are the x_j of Table 2's caption).
 *   Y       device FP32 [B, n], non-negative targets.
 *   W       device FP32 [B, kdim]: output weights; read as the start when
 *           p->warm == 1.
 *   logU    device FP32 [B, n] or NULL: output log of the source scaling u.
 *   logV    device FP32 [B, n]: output log of the target scaling v; read as
 *           the start when p->warm == 1.
 *   iters   device int32 [B] or NULL: iterations each spectrum took over
 *           both phases (the stopping test runs every check_every
 *           iterations).
 *   status  device int32 [B] or NULL: OTLM_S_* flags.
 * Each spectrum is frozen once its own test passes, so its result does not
 * depend on the other spectra of the batch.  The host thread blocks once per
 * `check_every` iterations to read the number of active spectra.
 * Errors: OTLM_E_INVALID (bad sizes or parameters: eps must equal the
 * kernel's, 1 <= kdim <= 256, B >= 0; negative or non-finite D or Y, or a D
 * column summing to 0), OTLM_E_UNSUPPORTED (WSTEP_EXACT beyond its sizes,
 * REFINE_FP64 without WSTEP_EXACT), OTLM_E_NOMEM, OTLM_E_HIP.  B = 0 is a
 * no-op.  A BF16 bulk phase keeps the state in FP32 and rounds only the
 * operands of the two kernel products (v, u and K) to BF16. */
int otlm_solve_batch(otlm_kernel k, const float* D, int64_t kdim, const float* Y, int64_t B,
                     const otlm_params* p, float* W, float* logU, float* logV,
                     int32_t* iters, int32_t* status, void* stream);

/* FP64 objective and optimality residuals at (W, logU, logV), per spectrum
 * (eq. OTLM in the scaling form eps KL(Q||K) + F1(Q1) + F2(Q^T 1) and its
 * Fenchel dual).  out is device FP64 [B, 6]:
 *   [0] primal  eps KL(Q||K) + lambda L(Q^T 1|y) + alpha R(w),  Q = diag(u) K diag(v)
 *   [1] dual    -F1*(-f) - F2*(-g) - eps sum_ij K_ij (e^{(f_i+g_j)/eps} - 1),
 *               f = eps log u, g = eps log v  (NaN for POISSON and BALANCED; for
 *               L1 / NONE the indicator F1* counts as 0 and feasibility
 *               D^T f >= -alpha shows in [5])
 *   [2] <C, Q>  transport cost (needs C: pass the same C as to make_kernel)
 *   [3] ||Q1 - Dw||_1 / ||Dw||_1
 *   [4] max_j dist(-g_j, dF2(m_j)) / lambda,  m = Q^T 1
 *   [5] max_j |min(w_j, alpha R'(w_j) + eps (D^T log u)_j)|
 * C is device FP64 [n, n].  Errors as otlm_solve_batch. */
int otlm_objective(otlm_kernel k, const double* C, const float* D, int64_t kdim, const float* Y,
                   int64_t B, const otlm_params* p, const float* W, const float* logU,
                   const float* logV, double* out, void* stream);

/* Kernel timing on the solve's own stream.  While enabled, otlm_solve_batch
 * brackets every launch of its hot kernels with HIP events and accumulates
 * their durations per kernel class (12 classes):
 *   [0] s = K v product, FP32 (+ log-ratio epilogue)
 *   [1] weight step, FP32 state: the MM GEMM epilogue (WSTEP_MM) or the
 *       Newton prox kernel (WSTEP_EXACT)
 *   [2] a = D w, u = a / s, FP32        [3] t = K^T u product + prox, FP32
 *   [4] convergence test
 *   [5]..[8] the same as [0]..[3] in the FP64 refinement phase
 *   [9] s = K v product in BF16 (FP32 accumulate)  [10] t = K^T u in BF16
 *   [11] MM warm-up steps of an exact-prox solve (cold starts, fallbacks)
 * otlm_profile_read copies the mean duration in ms per launch (ms[12]) and the
 * launch counts (count[12]) accumulated since the last enable, synchronising
 * the recorded events first, and the work the weight-prox kernels performed,
 * summed over spectra (newton_iters[6]: Newton iterations of the FP32-state
 * and FP64-state kernels, then their Hessian factorisations, then the
 * lower-triangle entries m (m + 1) / 2 of the free-set Hessians they built,
 * m the number of free weights; a profiled solve synchronises its stream at
 * the end to collect them).  Any output pointer
 * may be NULL.  Enabling resets the counters.  Errors: OTLM_E_INVALID for a
 * null kernel. */
int otlm_profile_enable(otlm_kernel k, int32_t on);
int otlm_profile_read(otlm_kernel k, double* ms, int64_t* count, int64_t* newton_iters);

/* ---------------------------------------------------------------------------
 * Ragged batches: spectra of different lengths, each with its own dictionary.
 *
 * Every spectrum b lives on the grid of one of `nkernels` Gibbs kernels
 * (kernel_of[b]), so n_b = that kernel's n, and has its own dictionary D_b
 * [n_b, kdim[b]] (the paper's X for that target).  All of them run Algorithm 1
 * together: the kernel products of the spectra that share a kernel form one
 * GEMM, and the products of all kernels are issued as one grouped launch per
 * step; the dictionary work (Table 2 MM step, a = D_b w, u = a / s) is one
 * fused workgroup per spectrum.  The weight step is the MM step of Table 2,
 * taken p->inner_max times per outer iteration at the same s = K v (every
 * repetition majorizes the same ProxP problem, so the limit is the one of
 * the single step; more repetitions cut the number of kernel products), and
 * for the spectra still active after opts->newton_after iterations the exact
 * weight prox (ProxP minimised by active-set Newton): MM steps crawl where
 * small weights sit under large overlapping peaks.
 * FP32 state and products (OTLM_PREC_FP32, OTLM_WSTEP_MM, no refinement).
 *
 * Packed arrays (device, FP32, in input order b = 0..B-1, no padding):
 *   D      D_0, D_1, ... each [n_b, kdim[b]] row-major     (sum n_b kdim[b])
 *   Y      y_0, y_1, ...      each [n_b]                   (sum n_b)
 *   logU, logV                 same layout as Y
 *   W      w_0, w_1, ...      each [kdim[b]]               (sum kdim[b])
 * ------------------------------------------------------------------------- */
typedef struct otlm_ragged_s* otlm_ragged;

typedef struct {
  int32_t use_graph;   /* 1 (default): each interval of check_every iterations
                          and its convergence test are captured once as a HIP
                          graph and replayed; 0: the same launches, eager     */
  int32_t tile;        /* -1 (default): time the four GEMM tile shapes of the
                          grouped kernel products (128x128, 128x64, 64x128,
                          64x64) on the plan's own shapes at create and keep
                          the fastest; 0..3: use that shape                  */
  int32_t newton_after;/* 15 (default): a spectrum with kdim <= 128 and
                          n <= 2048 still active after this many iterations
                          takes the exact weight prox (active-set Newton, as
                          OTLM_WSTEP_EXACT; FP64 Hessian for kdim <= 64, FP32
                          above) instead of MM steps; -1: MM only             */
  int32_t reserved;    /* set to 0                                            */
} otlm_ragged_opts;

/* use_graph = 1, tile = -1, newton_after = 15. */
void otlm_ragged_default_opts(otlm_ragged_opts* o);

/* Plan a ragged solve.
 *   kernels    host array [nkernels] of kernel objects (1 <= nkernels <= 8,
 *              n <= 4096 each, eps equal to p->eps); they must outlive the
 *              plan, which reads their K.
 *   kernel_of  host int32 [B]: kernel index of spectrum b.
 *   kdim       host int32 [B]: dictionary columns of spectrum b, 1..256.
 *   B          1 .. 2^22 spectra.
 *   p          parameters, fixed for the plan's lifetime; wstep must be
 *              OTLM_WSTEP_MM, prec OTLM_PREC_FP32, refine OTLM_REFINE_NONE;
 *              inner_max (1..64) is the number of MM steps per iteration.
 *   opts       NULL for the defaults.
 * Allocates the plan's device state (about 5 sum(np_b) + sum(n_b kdim[b])
 * floats), runs the tile timing and the graph capture, and synchronises
 * `stream`.  Errors: OTLM_E_INVALID, OTLM_E_UNSUPPORTED (other precision or
 * weight-step modes, n > 4096), OTLM_E_NOMEM, OTLM_E_HIP. */
int otlm_ragged_create(const otlm_kernel* kernels, int32_t nkernels, const int32_t* kernel_of,
                       const int32_t* kdim, int64_t B, const otlm_params* p,
                       const otlm_ragged_opts* opts, void* stream, otlm_ragged* out);

/* Solve the planned batch for the packed D and Y (layout above).  W and logV
 * are outputs, read as the start when p->warm == 1; logU, iters and status
 * (int32 [B], input order) may be NULL.  Copies D (transposed) and Y into the
 * plan, so they may change between calls.  Blocks the host once at the start
 * (input validation) and once per check interval (active count).
 * Errors: OTLM_E_INVALID (null arrays, called on another device than the
 * plan's, negative or non-finite D or Y, a D column summing to 0),
 * OTLM_E_HIP. */
int otlm_ragged_solve(otlm_ragged r, const float* D, const float* Y, float* W, float* logU,
                      float* logV, int32_t* iters, int32_t* status, void* stream);

/* Chosen tile (tile_bm x tile_bn), the timing of the four candidates in ms
 * (tune_ms[4], 0 when a tile was forced) and sizes[4] = {sum n_b, sum kdim[b],
 * sum n_b kdim[b], device bytes held by the plan}.  Any output may be NULL. */
int otlm_ragged_info(otlm_ragged r, int32_t* tile_bm, int32_t* tile_bn, double* tune_ms, int64_t* sizes);

/* Kernel timing of ragged solves, as otlm_profile_*, with 5 classes:
 * [0] grouped s = K v products  [1] per-spectrum weight step  [2] grouped
 * t = K^T u products with the target prox  [3] convergence test
 * [4] Newton weight prox.  While
 * enabled the solve launches eagerly (no graph replay) and counts the
 * algorithmic work of the timed launches into work[3] (may be NULL):
 * [0] multiply-adds of the kernel products, sum over launches and active
 * spectra of n_b^2 (both products); [1] bytes of the weight steps, per active
 * spectrum 4 (4 n_b + band entries of D_b + 2 kdim[b]); [2] flops of the
 * Newton weight prox, per Newton iteration 6 n_b kdim[b] (evaluation,
 * gradient, one trial point) plus 2 n_b per lower-triangle entry of the
 * free-set Hessians built.  Reading synchronises
 * the device. */
int otlm_ragged_profile_enable(otlm_ragged r, int32_t on);
int otlm_ragged_profile_read(otlm_ragged r, double* ms, int64_t* count, int64_t* work);

/* Release a plan.  NULL is a no-op.  Synchronises the device. */
int otlm_ragged_free(otlm_ragged r);

/* ---------------------------------------------------------------------------
 * Warm-start network (not part of the paper): a multilayer perceptron
 *   x -> GELU(x W1^T + b1) -> GELU(. W2^T + b2) -> . W3^T + b3
 * (exact erf GELU, weights [out, in] row-major, flat parameter vector
 * [W1, b1, W2, b2, W3, b3]) that maps a target spectrum y to a starting point
 * of Algorithm 1, the (log u, log v, w) the solver reaches for it.  Inputs are
 * standardised per feature and targets per output (after clamping to
 * [-50, 50]) with statistics of the training set; the loss is the (weighted)
 * mean squared error of the standardised outputs.  Trained by AdamW on minibatches of a
 * training set held in device memory; FP32 training, FP32 or BF16 inference.
 * ------------------------------------------------------------------------- */
typedef struct otlm_mlp_s* otlm_mlp;

typedef struct {
  double lr;            /* learning rate, >= 0                       */
  double beta1, beta2;  /* moment decays, in [0, 1)                  */
  double eps;           /* > 0                                       */
  double weight_decay;  /* decoupled decay on every parameter, >= 0  */
} otlm_adamw;

/* Create a network with layer widths dims[4] = {in, h1, h2, out} (in, h1, h2
 * multiples of 32; out a multiple of 16) and initial parameters theta (host or
 * device FP32, [nparam], copied).  Standardisation starts as the identity.
 * Synchronises `stream`.  Errors: OTLM_E_INVALID, OTLM_E_NOMEM, OTLM_E_HIP. */
int otlm_mlp_create(const int32_t* dims, const float* theta, void* stream, otlm_mlp* out);

/* Layer widths, parameter count and AdamW steps taken (any may be NULL). */
int otlm_mlp_info(otlm_mlp m, int32_t* dims, int64_t* nparam, int64_t* step);

/* Set the standardisation from a training set: X device FP32 [N, in] (raw
 * targets y), T device FP32 [N, out] (raw outputs, clamped to [-50, 50]);
 * per column mean and standard deviation (floored at 1e-6), FP64 sums.
 * Synchronises `stream`. */
int otlm_mlp_set_norm(otlm_mlp m, const float* X, const float* T, int64_t N, void* stream);

/* Loss weight omega_o >= 0 of every output (host or device FP32 [out]; the
 * default is 1): the loss is 1/(B out) sum_b sum_o omega_o (z_bo - t_bo)^2.
 * Synchronises `stream`.  Errors: OTLM_E_INVALID for a negative or non-finite
 * weight. */
int otlm_mlp_set_loss_weights(otlm_mlp m, const float* weights, void* stream);

/* Set the standardisation statistics directly (host or device FP32 [in] and
 * [out]; standard deviations > 0), e.g. to restore a saved network.
 * Synchronises `stream`. */
int otlm_mlp_set_norm_stats(otlm_mlp m, const float* in_mu, const float* in_sd, const float* out_mu,
                            const float* out_sd, void* stream);

/* Copy the standardisation statistics out (any pointer may be NULL). */
int otlm_mlp_get_norm(otlm_mlp m, float* in_mu, float* in_sd, float* out_mu, float* out_sd, void* stream);

/* Gradient of the loss on the minibatch of rows idx[0..B) (device int32) of X
 * [*, in] and T [*, out] (B a multiple of 16): grad device FP32 [nparam]
 * (may be NULL), loss device FP32 [1] (may be NULL).  No parameter update. */
int otlm_mlp_grad(otlm_mlp m, const float* X, const float* T, const int32_t* idx, int64_t B,
                  float* grad, float* loss, void* stream);

/* One AdamW step on the minibatch (as otlm_mlp_grad, then the update). */
int otlm_mlp_train_step(otlm_mlp m, const float* X, const float* T, const int32_t* idx, int64_t B,
                        const otlm_adamw* h, float* loss, void* stream);

/* Copy the parameters out / in (device or host FP32 [nparam]). */
int otlm_mlp_get_params(otlm_mlp m, float* theta, void* stream);
int otlm_mlp_set_params(otlm_mlp m, const float* theta, void* stream);

/* Predict starting points for B raw targets Y (device FP32 [B, in]) in
 * precision prec (OTLM_PREC_FP32, or OTLM_PREC_BF16: BF16 weights and
 * activations, FP32 accumulation).  The outputs are split by column: the first
 * n_u into logU [B, n_u] (may be NULL), the next n_v into logV [B, n_v], the
 * rest into W [B, out - n_u - n_v], clamped to >= 0, so logV and W can be
 * passed to otlm_solve_batch with warm = 1. */
int otlm_mlp_infer(otlm_mlp m, const float* Y, int64_t B, int32_t prec, int32_t n_u, int32_t n_v,
                   float* logU, float* logV, float* W, void* stream);

/* Release the network.  NULL is a no-op.  Synchronises the device. */
int otlm_mlp_free(otlm_mlp m);

/* Static description of an otlm_status code. */
const char* otlm_status_str(int code);

#ifdef __cplusplus
}
#endif
#endif /* OTLM_H */
