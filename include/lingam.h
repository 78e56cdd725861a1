/*
 * lingam.h -- C ABI of the MI355X (gfx950) DirectLiNGAM causal-order search.
 *
 * The library finds the causal order K of a linear non-Gaussian acyclic model
 * from observational data, the first (order-finding) step of DirectLiNGAM
 * that ParaLiNGAM accelerates (Shahbazinia, Salehkaleybar, Hashemi,
 * "ParaLiNGAM", arXiv 2109.13993):
 *   - Alg. 1 / Alg. 3: p iterations of: find the root, append it to K,
 *     remove it from U, regress it out of the remaining variables;
 *   - Alg. 2: the root is the variable of minimum score
 *     S_i = sum_j min(0, I(x_i, x_j, r_i^(j), r_j^(i)))^2, with the
 *     likelihood-ratio test of Eq. (Itest) and the entropy approximation of
 *     Eq. (HApp); this library reports T_i = -S_i (root = argmax T);
 *   - Sec. 3.1 (messaging): each unordered pair is evaluated once and the
 *     reverse test is its exact negation;
 *   - Sec. 3.2-3.3 (threshold): variables whose partial score exceeds a
 *     threshold gamma stop comparing; gamma is multiplied by c until the
 *     iteration can end.  The order is the same as without the threshold;
 *   - Sec. 3.4 (Eq. var_update, Eq. CovUpdate, UpdateData, UpdateCovMat):
 *     normalisation once, covariance once, then rank-1 updates of the data
 *     and of the covariance after every root.
 *
 * Every symbol is extern "C".  No C++ exception crosses the ABI.  All calls
 * are synchronous: they return once the results are in the caller's host
 * arrays.  Sizes are in elements unless stated otherwise.
 */
#ifndef LINGAM_H
#define LINGAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lingam_status {
  LINGAM_OK = 0,
  LINGAM_E_INVALID = 1,     /* bad argument: null pointer, n < 2, p < 1, size overflow,
                               wrong struct_size, forced order not a prefix of a permutation */
  LINGAM_E_NONFINITE = 2,   /* NaN or Inf in X (result.bad_i = variable) */
  LINGAM_E_DEGENERATE = 3,  /* a row of zero variance (bad_i), or a pair of remaining
                               variables with 1 - corr^2 <= 1e-12 (bad_i, bad_j), checked for
                               every pair at the start of each iteration, pruned or not: the
                               residual cannot be normalised */
  LINGAM_E_NOMEM = 4,       /* device allocation failed or the caller's workspace is too small */
  LINGAM_E_DEVICE = 5,      /* HIP runtime error; lingam_last_error() holds the text */
  LINGAM_E_UNSUPPORTED = 6  /* option combination not supported */
} lingam_status;

/* Arithmetic of the per-sample entropy reductions (the hot path), and of
 * the stored rows (Sec. 3.4 keeps the normalised data and its covariance).
 *   FP64 : everything in binary64.
 *   MIXED: the per-sample log cosh / exp terms in binary32 on the hardware
 *          exp2/log2 units, summed in binary32 over at most 32 samples per lane
 *          and then in binary64; residuals are formed in binary64 and then
 *          rounded; normalisation, covariance, regression coefficients,
 *          rank-1 updates and score sums stay binary64.
 *   FP32_STORAGE: MIXED with the normalised rows stored in binary32 (half the
 *          memory and traffic): residuals are formed by binary32 fused
 *          multiply-adds from the stored rows and b rounded to binary32; the
 *          covariance (of the stored rows), b, 1/sqrt(1 - b^2), the rank-1
 *          updates (rounded once when stored) and the score sums stay binary64.
 *          T_err_bound adds the residuals' input error.  Each iteration's rows
 *          are re-rounded, so the data drift from the binary64 path by about
 *          u32 per update; the bound covers one iteration on its stored rows. */
typedef enum lingam_precision {
  LINGAM_PREC_FP64 = 0,
  LINGAM_PREC_MIXED = 1,
  LINGAM_PREC_FP32_STORAGE = 2
} lingam_precision;

/* Layout of X.  VAR_MAJOR is the paper's p x n matrix, row i = the n samples
 * of variable i (Alg. 1 input).  SAMPLE_MAJOR is n x p, row k = sample k. */
typedef enum lingam_layout { LINGAM_LAYOUT_VAR_MAJOR = 0, LINGAM_LAYOUT_SAMPLE_MAJOR = 1 } lingam_layout;

/* How the tests of an iteration are mapped onto the GPU (opts.pair_strategy).
 * DEFAULT is this library's pair kernel.  The other three are the baseline
 * mappings the paper compares against (Sec. 5.3), kept as ablation
 * variants: they compute the same tests (every ordered pair, FP64, without
 * the threshold and without messaging) with a different parallel layout.
 *   BLOCK_WORKER   one work-group per variable; its tests one after another,
 *                  each over all samples with the whole work-group;
 *   THREAD_WORKER  one work-group per variable; each thread one test, the
 *                  thread walking all samples of its pair alone;
 *   BLOCK_COMPARE  one work-group per ordered pair of variables. */
typedef enum lingam_pair_strategy {
  LINGAM_PAIR_DEFAULT = 0,
  LINGAM_PAIR_BLOCK_WORKER = 1,
  LINGAM_PAIR_THREAD_WORKER = 2,
  LINGAM_PAIR_BLOCK_COMPARE = 3
} lingam_pair_strategy;

typedef struct lingam_opts {
  uint32_t struct_size;        /* must be sizeof(lingam_opts) */
  int32_t precision;           /* lingam_precision, default FP64 */
  int32_t layout;              /* lingam_layout, default VAR_MAJOR */
  int32_t x_dtype;             /* 0 = double, 1 = float; default 0 */
  int32_t x_on_device;         /* 1 = X is a device pointer on `device`, 0 = host pointer */
  int32_t device;              /* HIP device ordinal; -1 = the current device */
  int32_t use_threshold;       /* 1 = threshold early exit (default), 0 = evaluate every pair */
  double gamma0;               /* > 0: initial threshold of every iteration; <= 0 (default):
                                  adaptive, 1e-6 for the first iteration and then 1.5 times
                                  the previous iteration's root score (any value gives the same
                                  order; it only changes how many pairs are evaluated) */
  double gamma_mult;           /* threshold multiplier c; <= 1 selects 4 */
  int32_t cov_refresh_every;   /* k > 0: recompute the correlation matrix from the updated data
                                  every k iterations (FP64 matrix cores), the rank-1 UpdateCovMat
                                  recursion in between; 0 = the recursion only; < 0 (default): 1
                                  in FP64 mode, 16 in MIXED and FP32_STORAGE modes */
  int32_t max_roots;           /* 0 = full order; m > 0 = stop after m roots */
  const int32_t* forced_order; /* optional host array: follow these roots for the first
                                  forced_len iterations (scores are still computed) */
  int32_t forced_len;
  int32_t record_M_iters;      /* record the full test matrix for the first k iterations */
  int32_t band_blocks;         /* tuning: the threshold rounds compare every variable still below
                                  the threshold with bands of target blocks (8 variables each),
                                  refreshing the threshold state after each band.  0 (default): a
                                  first band of 4 blocks (single MIXED search) or 1 block (FP64,
                                  batches), then bands sized from the number of variables still
                                  below the threshold; k > 0: k blocks per band */
  int32_t chunk_samples;       /* tuning: samples per work-group chunk (multiple of 256), 0 = auto */
  void* stream;                /* hipStream_t to run on; NULL = a library-owned stream */
  int32_t profile;             /* 1 = time every pair-kernel launch with HIP events on the
                                  stream (fills seconds_pair_kernel / pair_kernel_launches) */
  void* workspace;             /* optional caller-owned device memory on `device` (e.g. from the
                                  PyTorch allocator), 256-byte aligned, that the call carves every
                                  device buffer from instead of allocating; NULL (default) = one
                                  allocation of the library per call.  It must hold at least
                                  lingam_workspace_size() (lingam_workspace_size_batch() for a
                                  batch) bytes, else the call returns LINGAM_E_NOMEM before any
                                  device work.  Not retained after the call returns; calls that
                                  share one workspace must not overlap. */
  uint64_t workspace_bytes;    /* size of `workspace` in bytes */
  int32_t estimate_B;          /* 1 = after the order, estimate the causal strengths B into
                                  result.B (Alg. 1, last step); needs the full order
                                  (max_roots 0) and p <= 8000 */
  int32_t batch_queue;         /* batches: 1 (default) = the pair work of every data set on one
                                  device work queue served by a persistent grid (finished or small
                                  sets occupy no work-groups); 0 = one grid slice per set.  Score
                                  rows run in grid slices either way */
  int32_t graph;               /* batches: 1 = capture each window of 16 iterations into a HIP graph
                                  and replay it; instantiated graphs are kept for later calls with
                                  device memory at the same address and of the same layout (pass the
                                  same opts.workspace).  0 (default) = launch kernel by kernel */
  double band_target;          /* tuning: pair-samples (alive rows x targets x n) that a later
                                  threshold band of round 0 aims at; <= 0 (default) = 6e7
                                  max(1, (p/1000)^4), at most 1.6e9, for a single MIXED /
                                  FP32_STORAGE search, 2e7 otherwise */
  int32_t first_band_blocks;   /* tuning: target blocks of an iteration's first threshold band, the
                                  later bands sized as by default (band_blocks = 0); 0 (default) = 4
                                  for a single MIXED / FP32_STORAGE search, 1 otherwise */
  int32_t messaging;           /* 1 (default) = each unordered pair evaluated once, the reverse test
                                  its exact negation (Sec. 3.1 messaging); 0 = every variable
                                  evaluates its own tests, each pair once per direction (the
                                  ablation without messaging: the same results, twice the pairs) */
  int32_t pair_strategy;       /* lingam_pair_strategy, default DEFAULT.  The baseline strategies
                                  need precision FP64, use_threshold = 0 and messaging = 0 (else
                                  INVALID) and run in lingam_fit_order and lingam_fit_order_noalloc
                                  (batches: UNSUPPORTED); results equal the default's up to the
                                  order in which sample terms are summed */
} lingam_opts;

/* Outputs.  All arrays are host memory owned by the caller; NULL = not wanted. */
typedef struct lingam_result {
  int32_t* order;       /* [p], required: order[t] = original index of the t-th root;
                           -1 past the last root produced */
  double* T;            /* [p*p]: T[t*p + v] = -S_v at iteration t (NaN if v not in U_t) */
  uint8_t* T_state;     /* [p*p]: 0 = v not in U_t, 1 = complete score, 2 = pruned by the
                           threshold (partial score: T is an upper bound of the full one) */
  double* H;            /* [p*p]: H[t*p + v] = entropy estimate of variable v at iteration t */
  double* M;            /* [record_M_iters*p*p]: M[t*p*p + i*p + j] = I(x_i, x_j, ...) at
                           iteration t; NaN where not evaluated */
  double* T_err_bound;  /* [p*p], MIXED precision: a-priori bound on |T - T_exact| of the
                           entry T[t*p + v] from binary32 rounding (per-sample terms, hardware
                           exp2/log2, lane sums), given the same data; 0 in FP64 mode, NaN
                           where T is NaN.  When the two largest T of an iteration differ by
                           more than the sum of their bounds, the root is the exact one. */
  double* B;            /* [p*p] with opts.estimate_B: B[i*p + j] = causal strength of x_j on
                           x_i, the least-squares coefficient of x_j when x_i is regressed
                           (with an intercept) on every variable before it in the order; 0
                           where x_j does not precede x_i */
  double* T_err_prob;   /* [p*p], mixed modes: a probable bound on |T - T_exact| beside the
                           worst-case T_err_bound: the rounding errors taken as independent
                           and zero-mean (Hoeffding, failure probability 2.5e-14 per entropy
                           estimate) plus the hardware exp2/log2 systematic error; 0 in FP64
                           mode, NaN where T is NaN */
  uint64_t pairs_evaluated;   /* unordered pairs whose test was needed and evaluated */
  uint64_t pair_samples;      /* pairs_evaluated x n (the throughput unit) */
  uint64_t pairs_computed;    /* pairs actually run by the kernel (>= pairs_evaluated) */
  uint64_t threshold_rounds;  /* threshold rounds over all iterations */
  uint64_t bands;             /* band launches over all iterations */
  double seconds_total;       /* wall time of the call */
  double seconds_device;      /* device time from the first to the last kernel */
  double seconds_pair_kernel; /* summed duration of the pair-kernel launches (opts.profile) */
  uint64_t pair_kernel_launches;  /* pair-kernel launches (counted when opts.profile) */
  int32_t iterations;         /* roots placed in order[] */
  int32_t bad_i, bad_j;       /* diagnostics for NONFINITE / DEGENERATE, else -1 */
  int32_t status;             /* lingam_status of this result (the per-set status of a batch) */
} lingam_result;

/* Fill *o with the defaults listed above (struct_size set). */
void lingam_opts_default(lingam_opts* o);

/*
 * Causal order of the p variables of X (n samples each).
 *   X   : p x n (VAR_MAJOR) or n x p (SAMPLE_MAJOR) array of x_dtype, host or
 *         device memory per opts->x_on_device; read only, not retained.
 *   o   : options, NULL = defaults.
 *   out : results (out->order required).
 * Returns LINGAM_OK or an error status; on error the order holds the roots
 * found so far.  Concurrent calls on different streams are allowed.
 */
lingam_status lingam_fit_order(const void* X, int64_t n, int64_t p, const lingam_opts* o,
                               lingam_result* out);

/* One data set of a batch: either its own X (sample_idx == NULL), or a
 * bootstrap resample of X given as n_idx sample indices (with repetitions)
 * into the n columns of X. */
typedef struct lingam_dataset {
  const void* X;
  int64_t n, p;
  const int64_t* sample_idx; /* host array of n_idx indices in [0, n), or NULL */
  int64_t n_idx;
} lingam_dataset;

/* Causal orders of `count` (<= 65535) independent data sets.  Every kernel
 * launch covers all sets of the batch at the same iteration (one descriptor
 * per set on the device), so many small searches share each launch; a set
 * whose iteration needs more threshold rounds than were queued leaves the
 * batch and is finished on its own.  The results are those of separate
 * lingam_fit_order calls with the same options: the same order, and bit for
 * bit the same T and T_err_bound entries wherever the score is complete in
 * both.  (A batch may schedule its threshold bands differently from a
 * single call, which changes only which variables end an iteration pruned,
 * their partial scores and the pair counters.)
 *   sets[k].X: host or device memory per opts->x_on_device, with opts->x_dtype
 *     and opts->layout; a bootstrap set (sample_idx != NULL) needs a binary64
 *     p x n base, its sample_idx is host memory, n_idx samples are drawn.
 *   outs[k]: as for lingam_fit_order (M unused); outs[k].status is that set's
 *     status.  forced_order and record_M_iters must be unset (UNSUPPORTED).
 * Returns LINGAM_OK if every set succeeded, else the status of the first set
 * that failed (the other results are still filled). */
lingam_status lingam_fit_order_batch(int32_t count, const lingam_dataset* sets,
                                     const lingam_opts* o, lingam_result* outs);

/* The same for one call of lingam_fit_order_batch over these data sets
 * (0 if the batch is invalid). */
uint64_t lingam_workspace_size_batch(int32_t count, const lingam_dataset* sets, const lingam_opts* o);

/*
 * lingam_fit_order for callers that cannot allocate device memory (code
 * under HIP graph capture of its own, tight serving loops, harnesses that
 * forbid hipMalloc).  Every device buffer of the call is carved from a fixed
 * 64 MiB device array that the library holds on each GPU it runs on until
 * the process ends; no device memory, stream or event is created, and the
 * search runs on opts->stream (NULL = the null stream).  Arguments, results
 * and errors are those of lingam_fit_order, plus:
 *   LINGAM_E_NOMEM if lingam_workspace_size(n, p, o) exceeds 64 MiB (e.g.
 *     p=100, n=10000 fits; p=500, n=20000 does not), before any device work;
 *   LINGAM_E_INVALID if opts->workspace is set, LINGAM_E_UNSUPPORTED if
 *     opts->profile is set (its timing events would allocate).
 * Calls on one GPU share its array, which keeps the last call's contents
 * (every buffer a search needs cleared is cleared by the search itself):
 * calls that overlap on one GPU race and must be serialised by the caller.
 */
lingam_status lingam_fit_order_noalloc(const void* X, int64_t n, int64_t p, const lingam_opts* o,
                                       lingam_result* out);

/* Device bytes one call of lingam_fit_order with these shape and options
 * uses (the workspace it allocates, or the least opts->workspace_bytes it
 * accepts); 0 for an invalid shape.  It depends on n, p, precision,
 * x_on_device, x_dtype, record_M_iters, forced_len and chunk_samples. */
uint64_t lingam_workspace_size(int64_t n, int64_t p, const lingam_opts* o);


/*
 * Alg. 1, last step: the causal strengths B of X from a given causal order
 * (Sec. 2.3: covariance-based least-squares regressions along the order).
 * Each variable is regressed, with an intercept, on every variable before
 * it in `order`; all regressions come from one binary64 Cholesky
 * factorisation of the input's correlation matrix permuted into the order.
 *   X     : as for lingam_fit_order (host or device, layout, dtype per opts)
 *   order : [p] host array, a permutation of 0..p-1 (roots first)
 *   B     : [p*p] host array, caller-owned: B[i*p + j] = coefficient of x_j in
 *           the regression of x_i, 0 where x_j does not precede x_i.
 * opts->precision chooses the stored rows the correlation is formed from
 * (binary32 rows for FP32_STORAGE); the factorisation is binary64 always.
 * Returns INVALID for a bad order or p > 8000, DEGENERATE (bad_i unset) if a
 * variable is a linear function of those before it. */
lingam_status lingam_estimate_B(const void* X, int64_t n, int64_t p, const int32_t* order,
                                const lingam_opts* o, double* B);

/* Measured error of the hardware binary32 exp2 and log2 (v_exp_f32,
 * v_log_f32) that the MIXED and FP32_STORAGE per-sample terms use, over every
 * binary32 argument of the ranges they take: exp2 on [-126, 0] (relative
 * error; below -126 the term is under 2^-126 absolutely) and log2 on [1, 2]
 * (absolute error), against the binary64 library functions.  Units of
 * u32 = 2^-24.  The rounding bound T_err_bound assumes exp2 within
 * LINGAM_EXP2_ERR and log2 within LINGAM_LOG2_ERR; lingam_check_terms lets a
 * caller (and the tests) confirm that on the device at hand. */
#define LINGAM_EXP2_ERR 2.0
#define LINGAM_LOG2_ERR 1.5
/* ... and the probable bound T_err_prob assumes their systematic error (the
 * largest mean error within one binade of the argument) within these.  On
 * MI355X the sweep measures exp2 within 1.42 (largest binade mean 0.52) and
 * log2 within 1.00 (mean -0.19). */
#define LINGAM_EXP2_BIAS 0.75
#define LINGAM_LOG2_BIAS 0.3
typedef struct lingam_term_check {
  double exp2_max_rel;          /* largest |exp2~(x) - 2^x| / 2^x */
  double exp2_mean_rel;         /* mean signed relative error over all arguments */
  double exp2_max_binade_mean;  /* largest |mean signed error| within one binade of |x| */
  double log2_max_abs;          /* largest |log2~(x) - log2 x| */
  double log2_mean_abs;         /* mean signed error */
  uint64_t exp2_count, log2_count;  /* arguments evaluated */
} lingam_term_check;

/* Run the sweep on `device` (-1 = the current one); about 1.1e9 + 8.4e6
 * evaluations. */
lingam_status lingam_check_terms(int32_t device, lingam_term_check* out);

/* Static text for a status code. */
const char* lingam_status_string(lingam_status s);

/* Detail text of the last error raised on the calling thread ("" if none). */
const char* lingam_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LINGAM_H */
