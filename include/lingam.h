/*
 * lingam.h -- C ABI of the MI355X (gfx950) DirectLiNGAM causal-ordering library.
 *
 * The library computes the causal-ordering search of DirectLiNGAM
 * (AcceleratedLiNGAM, arXiv 2403.03772, Section 2.2 and Algorithm 1): at each
 * step it standardizes the remaining residual columns, scores every pair with
 * the pairwise likelihood-ratio measure built on the maximum-entropy
 * approximation of differential entropy, accumulates the per-variable measure
 * k_i = sum_j min(0, R(i,j))^2, takes the most exogenous variable (largest
 * -k_i), and regresses it out of all the others (Section 2.2).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller unless a comment
 *     says "host".  The library never allocates device memory: callers pass a
 *     workspace sized by the matching *_workspace_size() query.
 *   - Sample matrices are FP32, row-major n x d with leading dimension
 *     ldx >= d (samples in rows, variables in columns: the dataset X[m, dim]
 *     of Algorithm 1).
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *   - Host-detectable errors (NULL pointer, bad size, workspace too small) are
 *     returned synchronously and enqueue nothing.  Errors the device detects
 *     (non-finite input, zero-variance column, collinear pair) are returned
 *     when the call synchronizes (LINGAM_FLAG_NO_SYNC not set), and are also
 *     copied to opts->dev_status when that pointer is given.
 *   - lingam_last_error() returns a thread-local message for the last
 *     non-OK status of the calling thread.
 *
 * Learned-proposal form (opts->proposer non-NULL): at every step with more
 * than learned_min_m active variables a small network (16 features ->
 * 128 -> 128 -> 1, ReLU, BF16 weights, FP32 accumulation) scores the active
 * variables, the exact measure k_i is computed only for the `topk` best
 * scored, and the choice is made as follows.  The candidates' rows bound every
 * other variable's k from below (sum over candidates c of max(0, R(c, l))^2),
 * and so do its pair measures against its eight most correlated non-candidate
 * variables ("witnesses": sum of min(0, R(l, w))^2), each column counted
 * once; the "suspects" are the variables whose bound does not exceed the best
 * candidate's k (with the FP64 resolution of near-ties, the default: its
 * near-tie limit k (1 + 4e-3) + 1e-12, and a near-tie among the measured rows
 * is decided in FP64 as the full step decides it; the row passes then choose
 * their own sample splits, while with LINGAM_FLAG_FP32_TIES they take the
 * full step's, so that every row they measure equals the full step's bit for
 * bit).  (a) No suspect: the best candidate is the plain search's choice
 * (certified).  (b) At most min(max_suspects, m/2 - topk) suspects:
 * the second pass first measures them against the `extension` variables
 * ranked right after the candidates (columns not yet counted), which raises
 * their bounds; the rows of those still at or below the best candidate's k
 * are then evaluated exactly, and the best of candidates and these suspects
 * is the plain choice.  (c) More: the best candidate is taken when
 * its score leads every non-candidate's by at least `margin`.  Otherwise, and
 * at every audit step (t % audit_every == 0, a check of the margin rule), the
 * full step of the exact search decides.  With margin = +inf the order is
 * the plain order.  This proposal layer is not part of the paper's method;
 * it is an addition on top of the exact search it accelerates.
 */
#ifndef LINGAM_MI355X_H
#define LINGAM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LINGAM_OK = 0,
  LINGAM_E_INVALID = -1,     /* bad argument (host check) or bad forced order */
  LINGAM_E_DEGENERATE = -2,  /* zero variance, |corr| >= 1 - 1e-12, non-finite data */
  LINGAM_E_HIP = -3,         /* a HIP runtime call failed */
  LINGAM_E_WORKSPACE = -4,   /* workspace NULL or smaller than required */
  LINGAM_E_UNSUPPORTED = -5  /* size beyond the supported range */
} lingam_status;

/* opts->flags */
#define LINGAM_FLAG_NO_SYNC 1u  /* return after enqueueing; device errors only via dev_status */
#define LINGAM_FLAG_GRAPH 2u    /* capture the whole call into one HIP graph, cache the
                                   instantiated graph per (jobs, buffers, workspace) and
                                   replay it on identical later calls */
#define LINGAM_FLAG_AUTOTUNE 4u /* time the pair kernels' launch shapes (sample split, waves
                                   per workgroup) on this call's data the first time its
                                   size bucket is seen (cached per process, and in the file
                                   named by the environment variable LINGAM_AUTOTUNE_CACHE
                                   if set) */
#define LINGAM_FLAG_FP32_TIES 8u /* decide near-ties from the FP32 measures alone (no FP64
                                    tie resolution; see lingam_causal_order) */

/* Per-call profile, filled when opts->profile is non-NULL (forces a sync). */
typedef struct lingam_profile {
  double total_ms;        /* enqueue-to-completion of the whole call, HIP events */
  double pair_ms;         /* summed duration of the all-pairs moment kernel launches */
  int64_t pair_launches;  /* number of those launches */
  double pair_evals;      /* sample-pair evaluations they performed (steps whose full
                             search ran): m (m - 1) n per step */
  double gram_ms;         /* duration of the Gram (correlation) kernel */
  double gram_flops;      /* algorithmic flops of that Gram: 2 * n * d * d */
  double resid_ms;        /* summed duration of the residualize kernels */
  double resid_bytes;     /* algorithmic HBM bytes of those: 28 * n * (m - 1) per step */
  double cand_ms;         /* learned form: summed duration of the candidate, extension
                             and suspect-row pair kernels */
  int64_t cand_launches;  /* ... its launches */
  double cand_evals;      /* ... its sample-pair evaluations (with the extension and
                             suspect-row passes): 2 K (m - 1) n per step, plus
                             2 n (suspects * extension + measured rows * (m - 1)) */
  int32_t tie_steps;      /* steps whose choice the FP64 tie resolution made */
  int32_t tie_rows;       /* ... rows it measured in FP64 */
  int32_t tie_overflow;   /* steps whose near-tied set held more than the 16 variables
                             the FP64 resolution takes (the FP32 measures decided) */
  int32_t reserved;       /* zero */
} lingam_profile;

/* Decisions of the learned form, summed over the jobs of a call (host). */
typedef struct lingam_learned_stats {
  int32_t learned_steps;  /* steps with a learned pass */
  int32_t certified;      /* ... whose best candidate was certified (audit and forced
                             steps included: the full step still decides those) */
  int32_t fallbacks;      /* ... decided by the full step because the margin was small */
  int32_t audits;         /* ... decided by the full step as audits */
  int32_t audit_agree;    /* audits whose full choice equalled the learned choice */
  int32_t suspects_max;   /* most non-candidates in one step whose lower bound did not
                             exceed the best candidate's k (0 = certified) */
  int64_t suspects_sum;   /* ... summed over learned steps */
  int32_t expanded;       /* steps decided exactly by the second pass */
  int32_t cleared;        /* ... of which the extension columns cleared every suspect */
  int64_t rows_sum;       /* suspects whose full rows the second pass measured */
} lingam_learned_stats;

/* The proposer network.  A proposer block is LINGAM_PROPOSER_SIZE FP32 values
 * (device): feature mean[16], feature scale[16] (inputs are (f - mean) /
 * scale), then LINGAM_PROPOSER_PARAMS trainable values W1[128][16], b1[128],
 * W2[128][128], b2[128], w3[128], b3. */
#define LINGAM_PROPOSER_FEATURES 16
#define LINGAM_PROPOSER_HIDDEN 128
#define LINGAM_PROPOSER_PARAMS 18817
#define LINGAM_PROPOSER_SIZE (32 + LINGAM_PROPOSER_PARAMS)

typedef struct lingam_opts {
  uint32_t struct_size;         /* sizeof(lingam_opts): ABI version check */
  uint32_t flags;               /* LINGAM_FLAG_* */
  const int32_t* forced_order;  /* device int32[forced_len] or NULL: at step t < forced_len
                                   take forced_order[t] instead of the argmax (teacher
                                   forcing / resume); measures are still computed */
  int32_t forced_len;           /* 0 .. d */
  int32_t reserved0;
  double* step_measures;        /* device double[(d-1) * d] or NULL: row t holds the measure
                                   -k_i of step t by original column id, NaN for columns
                                   already ordered */
  double* step_gap;             /* device double[d-1] or NULL: best minus runner-up measure */
  int32_t* dev_status;          /* device int32 or NULL: receives the device-side status */
  lingam_profile* profile;      /* HOST pointer or NULL: per-kernel timings (forces sync) */
  /* learned-proposal form (see the top of this file) */
  const float* proposer;        /* device FP32[LINGAM_PROPOSER_SIZE] or NULL: plain search */
  int32_t topk;                 /* most candidates per learned step: multiple of 8 in
                                   [8, 256]; a step with m variables takes about m/16 of
                                   them (a multiple of 8), at least min(32, topk);
                                   default 64 */
  int32_t audit_every;          /* full-step audit when t % audit_every == 0; 0 = never;
                                   default 0 (with margin = +inf every decision is
                                   already the exact one, so an audit only repeats it) */
  float margin;                 /* score lead that accepts the best candidate when the
                                   suspects are too many for the second pass; +inf never
                                   does (exact); default +inf */
  int32_t learned_min_m;        /* steps with m <= learned_min_m are plain; >= topk and
                                   >= 64; default 2 * topk */
  lingam_learned_stats* learned_stats; /* HOST pointer or NULL: filled when the call syncs */
  float* record_features;       /* device FP32[(d-1) * d * 16] or NULL: the 16 features of
                                   every active variable at every step, by step and original
                                   column id (training data); unwritten entries untouched */
  int32_t max_suspects;         /* most suspects the second pass evaluates (0 = no second
                                   pass); default 1024 */
  int32_t extension;            /* extension columns: the suspects are first measured
                                   against the variables ranked right after the
                                   candidates (this many; a multiple of 8 in [0, 256]),
                                   and only those whose bound still allows them to win
                                   have their full rows measured (single orderings
                                   only: a batched call with extension > 0 returns
                                   LINGAM_E_UNSUPPORTED); 0 = none (default:
                                   on the d = 1024 and 4096 workloads the suspects that
                                   survive the candidates and witnesses mostly survive
                                   the extension too, and its pass costs what it saves) */
  int32_t* step_log;            /* device int32[d] or NULL (learned form): per step, the low
                                   4 bits are 0 plain step, 1 learned choice, 2 full step
                                   (fallback or forcing), 3 audit, 4 decided by the suspect
                                   pass; bits 4..15 hold the step's suspect count and the
                                   bits from 16 up the suspects whose rows the second
                                   pass measured */
  int32_t waves_all;            /* launch shape: waves per workgroup of the all-pairs
                                   kernel (1, 2 or 4), 0 = the default or the autotuned
                                   choice; results do not depend on it */
  int32_t waves_rows;           /* ... of the learned form's candidate, extension and
                                   suspect row kernels */
} lingam_opts;

/* Fill *opts with defaults (no forcing, no extra outputs, plain search, synchronous). */
void lingam_opts_init(lingam_opts* opts);

/*
 * Workspace bytes needed by lingam_causal_order for an n x d problem.
 * Returns 0 for unsupported sizes (n < 2, d < 1, or beyond the supported
 * range).  `opts` may be NULL.
 */
size_t lingam_workspace_size(int64_t n, int64_t d, const lingam_opts* opts);

/*
 * DirectLiNGAM causal order of the d columns of X (Section 2.2 outer loop
 * around Algorithm 1).
 *   X      device FP32 [n x ldx] row-major, read only.
 *   order  device int32[d]: original column ids, most exogenous first.
 *   opts   optional (NULL = defaults).
 *   ws     device workspace of ws_bytes >= lingam_workspace_size(n, d, opts);
 *          its contents on entry do not matter, on exit they are undefined.
 * Ties of the measure go to the smallest original column id.  The pair
 * measures are computed in FP32 (FP64 when 64 or fewer variables remain);
 * when the best variable's k and others lie within 0.4% of each other at a
 * step (a near-tie that FP32 rounding could decide), their k are recomputed
 * in FP64 from the FP64 residuals and the choice follows those
 * (LINGAM_FLAG_FP32_TIES switches this off).
 * Returns LINGAM_OK or an error status (see the conventions above).
 */
int lingam_causal_order(const float* X, int64_t n, int64_t d, int64_t ldx, int32_t* order,
                        const lingam_opts* opts, void* ws, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): lingam_causal_order
 * without a workspace argument.  The workspace is a device array of
 * LINGAM_NOALLOC_SCRATCH_BYTES bytes inside the library, one per GPU the
 * library runs on, held until the process ends; the call itself allocates
 * nothing.
 *   Arguments and results as for lingam_causal_order.
 *   A size whose workspace (lingam_workspace_size(n, d, opts)) exceeds
 *   LINGAM_NOALLOC_SCRATCH_BYTES returns LINGAM_E_UNSUPPORTED (64 MiB holds,
 *   for example, d = 512 at n = 8192 or d = 256 at n = 16384); so do
 *   LINGAM_FLAG_GRAPH, LINGAM_FLAG_AUTOTUNE and a non-NULL opts->profile.
 * Every call on one GPU uses that GPU's array and leaves its contents behind
 * (the call initialises what it needs).  Calls that overlap in time on the
 * same GPU (several streams, several host threads, or a LINGAM_FLAG_NO_SYNC
 * call still running on another stream) race on the array; calls one after
 * another on one stream are safe.
 */
#define LINGAM_NOALLOC_SCRATCH_BYTES (64u << 20)
int lingam_causal_order_noalloc(const float* X, int64_t n, int64_t d, int64_t ldx,
                                int32_t* order, const lingam_opts* opts, void* stream);

/*
 * One job of a batched call: the causal order of d columns of a sample
 * matrix, optionally over a resampled set of its rows.
 *   X        device FP32 [n_rows x ldx] row-major, read only (jobs may share it).
 *   rows     device int32[n] or NULL: sample s of the job is row rows[s] of X
 *            (bootstrap resampling with replacement); NULL = rows 0 .. n-1.
 *            Indices outside [0, n_rows) make the job fail with
 *            LINGAM_E_INVALID.
 *   n, d     samples and variables of the job (n >= 2, d >= 1).
 *   order    device int32[d] output, as for lingam_causal_order.
 *   step_measures / step_gap  optional per-step outputs, as in lingam_opts.
 */
typedef struct lingam_job {
  const float* X;
  int64_t n_rows;
  int64_t ldx;
  const int32_t* rows;
  int64_t n;
  int64_t d;
  int32_t* order;
  double* step_measures;
  double* step_gap;
  float* record_features;  /* as in lingam_opts, per job, or NULL */
} lingam_job;

/* Workspace bytes for lingam_batch_causal_order (0 if a job is invalid). */
size_t lingam_batch_workspace_size(const lingam_job* jobs, int32_t n_jobs,
                                   const lingam_opts* opts);

/*
 * The causal orders of many independent jobs (bootstrap resamples, datasets
 * of uneven n and d) in one batched run: every kernel launch covers the
 * current step of all jobs still running, so small jobs fill the GPU
 * together (Section 2.2 search per job, unchanged).
 *   jobs        HOST array of n_jobs descriptors (device pointers inside).
 *   job_status  device int32[n_jobs] or NULL: per-job device status.
 *   opts        flags (LINGAM_FLAG_GRAPH, _AUTOTUNE, _NO_SYNC), profile and the
 *               learned-form fields (shared by all jobs); forcing and
 *               opts-level per-step outputs are rejected.
 * Returns the first failing job's status, or LINGAM_OK.  A degenerate job
 * does not stop the others.
 */
int lingam_batch_causal_order(const lingam_job* jobs, int32_t n_jobs, int32_t* job_status,
                              const lingam_opts* opts, void* ws, size_t ws_bytes,
                              void* stream);

/* Workspace bytes for lingam_residualize on an n x d matrix (0 if unsupported). */
size_t lingam_residualize_workspace_size(int64_t n, int64_t d);

/*
 * Remove the effect of variable `exo` from every other variable listed in
 * `active` by least squares (the DirectLiNGAM update of Section 2.2):
 *   x_v <- x_v - (cov(x_v, x_exo) / var(x_exo)) x_exo,
 * population (ddof = 0) moments, computed in FP64.  In place on X.
 *   X       device FP32 [n x ldx] row-major, modified in place (only the
 *           active columns other than exo change).
 *   active  device int32[n_active], distinct column ids in [0, d).
 *   exo     the regressor column id (host value, 0 <= exo < d).
 * Returns LINGAM_E_DEGENERATE (after a sync) if var(x_exo) == 0.
 */
int lingam_residualize(float* X, int64_t n, int64_t d, int64_t ldx, const int32_t* active,
                       int32_t n_active, int32_t exo, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for lingam_adjacency on n samples of d variables (0 if unsupported). */
size_t lingam_adjacency_workspace_size(int64_t n, int64_t d);

/*
 * Weighted adjacency matrix from a causal order: every variable is regressed
 * by least squares, with an intercept, on the variables that precede it in
 * `order` (DirectLiNGAM's second phase, described in Section 1; the model is
 * the linear structural equation of Section 2.2).
 *   X       device FP32 [n_rows x ldx] row-major, read only.
 *   rows    device int32[n] or NULL: sample s is row rows[s] of X (a
 *           bootstrap resample); NULL = rows 0 .. n-1 (then n <= n_rows).
 *   n, d    samples and variables.
 *   order   device int32[d], a permutation of 0 .. d-1, exogenous first.
 *   B       device double[d * d] row-major: B[i d + j] is the coefficient of
 *           x_j in the regression of x_i when x_j precedes x_i; 0 elsewhere
 *           (the diagonal, the first variable's row, all later variables).
 * FP64 throughout (the data are widened on load): centred covariance on FP64
 * MFMA, blocked Cholesky of it in the causal order, B = I - diag(L) L^-1.
 * Synchronizes.  Returns LINGAM_E_INVALID if `order` is not a permutation or
 * a row index is outside [0, n_rows), LINGAM_E_DEGENERATE for non-finite
 * data or a covariance that is not positive definite (collinear variables,
 * or n <= d).
 */
int lingam_adjacency(const float* X, int64_t n_rows, int64_t ldx, const int32_t* rows, int64_t n,
                     int64_t d, const int32_t* order, double* B, void* ws, size_t ws_bytes,
                     void* stream);

/* Workspace bytes for lingam_adjacency_pruned (0 if unsupported). */
size_t lingam_adjacency_pruned_workspace_size(int64_t n, int64_t d);

/*
 * Adjacency matrix pruned by the adaptive lasso (a reading of ours: the paper
 * stops at the regressions of lingam_adjacency).  For every variable y and
 * its order predecessors P, on standardized data (population moments): the
 * least-squares coefficients b give weights w = |b|; the lasso path of y on
 * the weighted predictors is followed by least angle regression with the
 * lasso modification (Efron et al. 2004) up to max_active active
 * predictors; the breakpoint of least BIC, n log(2 pi s2) + RSS/s2 +
 * log(n) df with s2 = RSS_ols / (n - |P| - 1) and df its nonzero count, is
 * kept; its predictors are refitted by least squares with an intercept.
 *   Arguments as for lingam_adjacency; max_active in [1, 64].
 *   B      device double[d * d]: the refitted coefficients of the kept
 *          predictors, 0 elsewhere.
 * FP64 throughout.  Synchronizes.  LINGAM_E_INVALID as for lingam_adjacency;
 * LINGAM_E_DEGENERATE for n <= d + 1, non-finite data or a correlation
 * matrix that is not positive definite.
 */
int lingam_adjacency_pruned(const float* X, int64_t n_rows, int64_t ldx, const int32_t* rows,
                            int64_t n, int64_t d, const int32_t* order, int32_t max_active,
                            double* B, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for lingam_total_effects (0 if unsupported). */
size_t lingam_total_effects_workspace_size(int64_t d);

/*
 * Total causal effects of the linear acyclic model x = B x + e (Section 2.2;
 * Section 4.2 ranks the variables by them): T = (I - B)^-1, T[i d + j] the
 * effect on x_i of a unit change of x_j along all directed paths, T[i d + i] =
 * 1.
 *   B      device double[d * d]: an adjacency along `order` (as from
 *          lingam_adjacency); entries not below the order's diagonal (x_j
 *          after x_i) are ignored.
 *   order  device int32[d], a permutation of 0 .. d-1.
 *   T      device double[d * d], must not alias B.
 * I - B is unit lower triangular in the order; its inverse is the blocked
 * FP64 MFMA triangular inverse.  Synchronizes once (the order check); a
 * non-permutation returns LINGAM_E_INVALID.
 */
int lingam_total_effects(const double* B, int64_t d, const int32_t* order, double* T, void* ws,
                         size_t ws_bytes, void* stream);

/*
 * Bootstrap statistics (resampling the rows, ordering and regressing each
 * resample): add one resample's result to running counts.
 *   order        device int32[d]: the resample's causal order (a permutation;
 *                entries outside [0, d) are skipped, never written through).
 *   B            device double[d * d]: its adjacency (lingam_adjacency).
 *   order_count  device int32[d * d]: [i d + j] += 1 when x_j precedes x_i.
 *   edge_count   device int32[d * d]: [i d + j] += 1 when |B[i d + j]| > threshold.
 *   coef_sum     device double[d * d] or NULL: += B.
 * Enqueued on `stream`; no sync.  Divided by the number of resamples, the
 * counts are the order and edge probabilities.
 */
int lingam_bootstrap_accumulate(const int32_t* order, const double* B, int64_t d,
                                double threshold, int32_t* order_count, int32_t* edge_count,
                                double* coef_sum, void* stream);

/*
 * Bootstrap probabilities from the counts of lingam_bootstrap_accumulate
 * after n_resamples resamples: order_prob[i d + j] = P(x_j precedes x_i),
 * edge_prob[i d + j] = P(|B[i d + j]| > threshold), coef_mean = coef_sum /
 * n_resamples (skipped when coef_sum is NULL; coef_mean may then be NULL).
 *   order_count, edge_count  device int32[d * d];  coef_sum  device double[d * d] or NULL.
 *   order_prob, edge_prob    device double[d * d] outputs;  coef_mean  device double[d * d].
 * Enqueued on `stream`; no sync.  n_resamples < 1 returns LINGAM_E_INVALID.
 */
int lingam_bootstrap_finalize(const int32_t* order_count, const int32_t* edge_count,
                              const double* coef_sum, int64_t d, int32_t n_resamples,
                              double* order_prob, double* edge_prob, double* coef_mean,
                              void* stream);

/*
 * Workspace bytes for varlingam_fit on a T x d series with `lags` lags
 * (0 if unsupported: d < 1, lags < 1, or T - lags <= 1 + lags * d).
 */
size_t varlingam_workspace_size(int64_t T, int64_t d, int32_t lags, const lingam_opts* opts);

/*
 * VarLiNGAM (Section 3.2): least-squares VAR(lags) with intercept, the
 * DirectLiNGAM causal order of its residuals, and the instantaneous matrix B0.
 *   X      device FP32 [T x ldx] row-major series (time in rows), read only.
 *   M      device double[lags * d * d] or NULL: M[(tau-1) d d + i d + j] is the
 *          coefficient of x_j(t - tau) in the equation of x_i(t).
 *   resid  device FP32 [(T - lags) x d] row-major or NULL: the VAR residuals.
 *   order  device int32[d]: causal order of the residuals, exogenous first.
 *   B0     device double[d * d] or NULL: B0[i d + j] is the least-squares
 *          coefficient of residual j when residual i is regressed (with
 *          intercept) on all residuals that precede i in `order`; 0 elsewhere.
 *   opts   as for lingam_causal_order (forcing and per-step outputs apply to
 *          the ordering of the residuals; n = T - lags there).
 * The VAR normal equations are formed on FP64 MFMA and solved by Cholesky in
 * FP64; the residuals stay FP64 for the ordering.  Returns LINGAM_E_DEGENERATE
 * if the normal equations are not positive definite.
 */
int varlingam_fit(const float* X, int64_t T, int64_t d, int64_t ldx, int32_t lags, double* M,
                  float* resid, int32_t* order, double* B0, const lingam_opts* opts, void* ws,
                  size_t ws_bytes, void* stream);

/*
 * Lagged effects of VarLiNGAM's structural model (Section 3.2): with the VAR
 * matrices M_tau and the instantaneous matrix B0 that varlingam_fit returns,
 * theta_tau = (I - B0) M_tau for tau = 1 .. lags (the model equation solved
 * for x(t) gives M_tau = (I - B0)^-1 theta_tau).
 *   M      device double[lags * d * d], layout of varlingam_fit's M.
 *   B0     device double[d * d].
 *   theta  device double[lags * d * d], same layout as M; must not alias M.
 * Enqueued on `stream`; no workspace, no sync.
 */
int varlingam_lagged_effects(const double* M, const double* B0, int64_t d, int32_t lags,
                             double* theta, void* stream);

/*
 * Proposer network (the learned-proposal form; its kernels are the ones the
 * ordering runs).  Features are FP32 [rows x 16] row-major, as recorded by
 * opts->record_features.
 */

/* Workspace bytes for lingam_proposer_scores. */
size_t lingam_proposer_scores_workspace_size(void);

/* scores[r] = network(features[r]) for r < rows (FP32 out, device). */
int lingam_proposer_scores(const float* proposer, const float* features, int64_t rows,
                           float* scores, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for lingam_proposer_grad (0 if rows < 1 or n_lists < 1). */
size_t lingam_proposer_grad_workspace_size(int64_t rows, int32_t n_lists);

/*
 * Listwise softmax cross-entropy of the network over n_lists lists and its
 * gradient.  List L is rows offsets[L] .. offsets[L+1]-1 (device int64,
 * non-decreasing from 0 to rows); its target is row targets[L] (device
 * int64, inside the list).  loss = mean over lists of
 * logsumexp(s_L) - s_target.
 *   grad    device FP32[LINGAM_PROPOSER_PARAMS]: d loss / d (trainable values),
 *           at the BF16-rounded weights the forward pass uses.
 *   loss    device FP32[1] or NULL.
 *   scores  device FP32[rows] or NULL: the forward scores.
 * Synchronizes; a malformed offsets / targets array returns LINGAM_E_INVALID.
 */
int lingam_proposer_grad(const float* proposer, const float* features, int64_t rows,
                         const int64_t* offsets, const int64_t* targets, int32_t n_lists,
                         float* grad, float* loss, float* scores, void* ws, size_t ws_bytes,
                         void* stream);

/*
 * As lingam_proposer_grad with a soft target per list: weights device
 * FP32[rows] >= 0; the target distribution of list L is its rows' weights
 * divided by their sum, and loss = mean over lists of
 * sum_r q_r (logsumexp(s_L) - s_r) (one-hot weights give the hard loss).
 * Uses the workspace of lingam_proposer_grad_workspace_size.  Synchronizes;
 * malformed offsets, a negative or non-finite weight, or a list whose weights
 * sum to 0 return LINGAM_E_INVALID.
 */
int lingam_proposer_grad_soft(const float* proposer, const float* features, int64_t rows,
                              const int64_t* offsets, const float* weights, int32_t n_lists,
                              float* grad, float* loss, float* scores, void* ws,
                              size_t ws_bytes, void* stream);

/*
 * One Adam step (bias-corrected; Kingma and Ba) on the trainable values of
 * `proposer` (the normalisation stays): m1, m2 device FP32[PARAMS] moment
 * buffers (zero before step 1), step >= 1.
 */
int lingam_proposer_adam(float* proposer, const float* grad, float* m1, float* m2, int32_t step,
                         float lr, float beta1, float beta2, float eps, void* stream);

/* Thread-local text of the last error of the calling thread ("" if none). */
const char* lingam_last_error(void);

/* Library version string. */
const char* lingam_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LINGAM_MI355X_H */
