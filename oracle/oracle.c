/*
 * oracle.c -- plain FP64 CPU definition of the DirectLiNGAM causal-order
 * search that ParaLiNGAM accelerates (Shahbazinia, Salehkaleybar, Hashemi,
 * "ParaLiNGAM", arXiv 2109.13993).
 *
 * TEST INFRASTRUCTURE ONLY.  This file states what the GPU library has to
 * compute so that the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark can check it.  The GPU library never links, loads or calls
 * it, and it shares no code, header or constant table with the GPU library.
 *
 * What is computed (all arithmetic in IEEE binary64):
 *   - Alg. 1 (DirectLiNGAM): repeat FindRoot, append the root to the causal
 *     order K, remove it from U and regress it out of the data.  Its final
 *     step (estimating B from K) is not part of this search.
 *   - Alg. 2 (FindRoot): for every ordered pair (i, j) of remaining
 *     variables, normalise x_i and x_j, regress each on the other, normalise
 *     both residuals and add min(0, I)^2 to the score of i; the root is the
 *     variable of minimum score.
 *   - Eq. (Itest): I(x_i, x_j, r_i^(j), r_j^(i)) =
 *         H(x_j) + H(r_i^(j)) - H(x_i) - H(r_j^(i)).
 *   - Eq. (HApp): H(u) ~ H(nu) - k1 (E[log cosh u] - beta)^2
 *                             - k2 (E[u exp(-u^2/2)])^2,
 *     H(nu) = (1 + log 2 pi)/2, k1 = 79.047, k2 = 7.4129, beta = 0.37457.
 *   - Sec. 3.4, definition of the residual: r_i^(j) = x_i - cov(x_i,x_j)/var(x_j) x_j;
 *     variances and covariances use the adjusted (n-1) divisor.
 *
 * Readings taken where the paper is silent or garbled:
 *   - E{.} in Eq. (HApp) is the plain sample mean (1/n) sum.
 *   - "Normalize" means subtract the sample mean and divide by the (n-1)
 *     standard deviation (the adjusted sample variance of Sec. 3.4).
 *   - The test is grouped as (H(x_j) + H(r_i^(j))) - (H(x_i) + H(r_j^(i))),
 *     so the reverse test is the exact negation (messaging, Sec. 3.1).
 *   - The loop of Alg. 1 runs until U is empty; the last variable is
 *     appended without a comparison (Alg. 2).
 *   - Ties in the minimum score go to the variable with the lowest original
 *     index (U keeps the original order).
 *   - A zero or non-finite row variance, or a residual variance <= 1e-12,
 *     is reported as a degenerate input instead of being divided by.
 *   - Scores are reported as T = -S (larger is better); the root is argmax T.
 *
 * Every sum is an FP64 Neumaier-compensated sum taken in sample order; each
 * ordered pair is evaluated on one thread, so results do not depend on the
 * number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_INVALID 1
#define OR_E_NONFINITE 2
#define OR_E_DEGENERATE 3
#define OR_E_NOMEM 4

/* Eq. (HApp) constants, as printed in the paper. */
static const double HAPP_K1 = 79.047;
static const double HAPP_K2 = 7.4129;
static const double HAPP_BETA = 0.37457;
static const double RESID_VAR_MIN = 1e-12;

/* ---- compensated summation (Neumaier) ---------------------------------- */
typedef struct { double s, c; } csum;
static inline void cs_add(csum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static inline double cs_val(const csum* a) { return a->s + a->c; }

static double mean_of(const double* x, int64_t n) {
  csum a = {0, 0};
  for (int64_t k = 0; k < n; ++k) cs_add(&a, x[k]);
  return cs_val(&a) / (double)n;
}

/* adjusted sample covariance, 1/(n-1) sum (x - mean x)(y - mean y) */
static double cov_of(const double* x, const double* y, int64_t n) {
  double mx = mean_of(x, n), my = mean_of(y, n);
  csum a = {0, 0};
  for (int64_t k = 0; k < n; ++k) cs_add(&a, (x[k] - mx) * (y[k] - my));
  return cs_val(&a) / (double)(n - 1);
}

/* Normalize: z = (x - mean) / sqrt(adjusted variance).  Returns a status.
 * `var_min` is the smallest variance accepted. */
static int normalize_row(const double* x, int64_t n, double* z, double var_min) {
  double mu = mean_of(x, n);
  csum a = {0, 0};
  for (int64_t k = 0; k < n; ++k) {
    double d = x[k] - mu;
    cs_add(&a, d * d);
  }
  double var = cs_val(&a) / (double)(n - 1);
  if (!isfinite(mu) || !isfinite(var)) return OR_E_NONFINITE;
  if (!(var > var_min)) return OR_E_DEGENERATE;
  double sd = sqrt(var);
  for (int64_t k = 0; k < n; ++k) z[k] = (x[k] - mu) / sd;
  return OR_OK;
}

/* log(cosh(u)) taken directly; beyond |u| = 700 cosh overflows, and there
 * log cosh u = |u| - log 2 to double precision. */
static inline double log_cosh(double u) {
  double a = fabs(u);
  if (a < 700.0) return log(cosh(a));
  return a - log(2.0);
}

/* Eq. (HApp) on a sample u[0..n) (expected to be standardized). */
double oracle_entropy(const double* u, int64_t n) {
  csum e1 = {0, 0}, e2 = {0, 0};
  for (int64_t k = 0; k < n; ++k) {
    cs_add(&e1, log_cosh(u[k]));
    cs_add(&e2, u[k] * exp(-u[k] * u[k] / 2.0));
  }
  double E1 = cs_val(&e1) / (double)n;
  double E2 = cs_val(&e2) / (double)n;
  double h_nu = 0.5 * (1.0 + log(2.0 * M_PI));
  double d1 = E1 - HAPP_BETA;
  return h_nu - HAPP_K1 * d1 * d1 - HAPP_K2 * E2 * E2;
}

/* Both sample moments of Eq. (HApp) (for pins that check them directly). */
void oracle_entropy_moments(const double* u, int64_t n, double* E1, double* E2) {
  csum e1 = {0, 0}, e2 = {0, 0};
  for (int64_t k = 0; k < n; ++k) {
    cs_add(&e1, log_cosh(u[k]));
    cs_add(&e2, u[k] * exp(-u[k] * u[k] / 2.0));
  }
  *E1 = cs_val(&e1) / (double)n;
  *E2 = cs_val(&e2) / (double)n;
}

int oracle_standardize(const double* x, int64_t n, double* z) {
  if (!x || !z || n < 2) return OR_E_INVALID;
  return normalize_row(x, n, z, 0.0);
}

/* Regress a on b (Sec. 3.4): r = a - cov(a,b)/var(b) b, then Normalize(r)
 * into out, and return H(out).  Status in *st. */
static double residual_entropy(const double* a, const double* b, int64_t n,
                               double* tmp, double* out, int* st) {
  double c = cov_of(a, b, n);
  double vb = cov_of(b, b, n);
  double coef = c / vb;
  for (int64_t k = 0; k < n; ++k) tmp[k] = a[k] - coef * b[k];
  *st = normalize_row(tmp, n, out, RESID_VAR_MIN);
  if (*st != OR_OK) return NAN;
  return oracle_entropy(out, n);
}

/* Compare (Alg. 2, the normalise/regress/normalise/test body) for one
 * ordered pair of already-normalised rows zi, zj with entropies hi, hj.
 * scratch holds 2n doubles. */
static int compare_normalized(const double* zi, const double* zj, double hi, double hj,
                              int64_t n, double* scratch, double* I_out, double* corr_out) {
  double* tmp = scratch;
  double* r = scratch + n;
  int st;
  if (corr_out) *corr_out = cov_of(zi, zj, n) / sqrt(cov_of(zi, zi, n) * cov_of(zj, zj, n));
  double h_ri = residual_entropy(zi, zj, n, tmp, r, &st); /* r_i^(j) */
  if (st != OR_OK) return st;
  double h_rj = residual_entropy(zj, zi, n, tmp, r, &st); /* r_j^(i) */
  if (st != OR_OK) return st;
  *I_out = (hj + h_ri) - (hi + h_rj); /* Eq. (Itest) */
  return OR_OK;
}

/* The test I(x_i, x_j, r_i^(j), r_j^(i)) for two raw rows. */
int oracle_compare(const double* xi, const double* xj, int64_t n, double* I_out) {
  if (!xi || !xj || !I_out || n < 2) return OR_E_INVALID;
  double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)n);
  if (!buf) return OR_E_NOMEM;
  double* zi = buf;
  double* zj = buf + n;
  int st = normalize_row(xi, n, zi, 0.0);
  if (st == OR_OK) st = normalize_row(xj, n, zj, 0.0);
  if (st == OR_OK) {
    double hi = oracle_entropy(zi, n), hj = oracle_entropy(zj, n);
    st = compare_normalized(zi, zj, hi, hj, n, buf + 2 * n, I_out, NULL);
  }
  free(buf);
  return st;
}

/* One FindRoot evaluation (Alg. 2) over the rows listed in U.
 *   Z    : p x n working data (rows of variables still in U are used)
 *   U    : r indices into Z, ascending
 *   S    : [r] out, scores (sum over j of min(0, I_ij)^2, ascending j)
 *   Mrow : optional, r x r out, Mrow[a*r+b] = I for the ordered pair (U[a], U[b]),
 *          NaN on the diagonal
 *   Brow : optional, r x r out, correlation of the normalised pair (NaN diagonal)
 *   only : optional [r] mask; when given, only rows with only[a] != 0 get
 *          scores (other S entries are NaN) -- used by sampled checks.
 * On a degenerate pair, bad_a and bad_b receive the positions in U. */
static int find_root_scores_once(const double* Z, int64_t n, const int32_t* U, int32_t r,
                                 const double* H, double* S, double* Mrow, double* Brow,
                                 int nthreads, int32_t* bad_a, int32_t* bad_b);

static int find_root_scores(const double* Z, int64_t n, const int32_t* U, int32_t r,
                            const double* H, double* S, double* Mrow, double* Brow,
                            const uint8_t* only, int nthreads, int32_t* bad_a, int32_t* bad_b,
                            int pair_once) {
  if (pair_once && !only)
    return find_root_scores_once(Z, n, U, r, H, S, Mrow, Brow, nthreads, bad_a, bad_b);
  int status = OR_OK;
  int32_t ba = -1, bb = -1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
  {
    double* scratch = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!scratch) {
#ifdef _OPENMP
#pragma omp critical
#endif
      status = OR_E_NOMEM;
    }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int32_t a = 0; a < r; ++a) {
      if (!scratch) continue;
      if (only && !only[a]) { S[a] = NAN; continue; }
      const double* zi = Z + (int64_t)U[a] * n;
      csum s = {0, 0};
      int local = OR_OK;
      if (Mrow) Mrow[(int64_t)a * r + a] = NAN;
      if (Brow) Brow[(int64_t)a * r + a] = NAN;
      for (int32_t b = 0; b < r; ++b) {
        if (b == a) continue;
        const double* zj = Z + (int64_t)U[b] * n;
        double I, corr;
        int st = compare_normalized(zi, zj, H[a], H[b], n, scratch, &I, Brow ? &corr : NULL);
        if (st != OR_OK) {
          local = st;
#ifdef _OPENMP
#pragma omp critical
#endif
          {
            if (status == OR_OK) { status = st; ba = a; bb = b; }
          }
          break;
        }
        if (Mrow) Mrow[(int64_t)a * r + b] = I;
        if (Brow) Brow[(int64_t)a * r + b] = corr;
        double m = I < 0.0 ? I : 0.0;
        cs_add(&s, m * m);
      }
      S[a] = local == OR_OK ? cs_val(&s) : NAN;
    }
    free(scratch);
  }
  if (bad_a) *bad_a = ba;
  if (bad_b) *bad_b = bb;
  return status;
}

/* The same scores with each unordered pair evaluated once (messaging,
 * Sec. 3.1): Compare of (b, a) evaluates the two residual entropies of
 * Compare of (a, b) with the roles swapped, and the grouping of Eq. (Itest)
 * makes its result the exact IEEE negation, so I_ba is taken as -I_ab.  The
 * scores are then summed exactly as above (ascending b), so every output is
 * bitwise the one of the ordered evaluation; only the work halves. */
static int find_root_scores_once(const double* Z, int64_t n, const int32_t* U, int32_t r,
                                 const double* H, double* S, double* Mrow, double* Brow,
                                 int nthreads, int32_t* bad_a, int32_t* bad_b) {
  int status = OR_OK;
  int32_t ba = -1, bb = -1;
  double* Mall = (double*)malloc(sizeof(double) * (size_t)r * (size_t)r);
  double* Ball = Brow ? (double*)malloc(sizeof(double) * (size_t)r * (size_t)r) : NULL;
  if (!Mall || (Brow && !Ball)) {
    free(Mall); free(Ball);
    return OR_E_NOMEM;
  }
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
  {
    double* scratch = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!scratch) {
#ifdef _OPENMP
#pragma omp critical
#endif
      status = OR_E_NOMEM;
    }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int32_t a = 0; a < r; ++a) {
      if (!scratch) continue;
      const double* zi = Z + (int64_t)U[a] * n;
      Mall[(int64_t)a * r + a] = NAN;
      if (Ball) Ball[(int64_t)a * r + a] = NAN;
      for (int32_t b = a + 1; b < r; ++b) {
        const double* zj = Z + (int64_t)U[b] * n;
        double I = NAN, corr = NAN;
        int st = compare_normalized(zi, zj, H[a], H[b], n, scratch, &I, Ball ? &corr : NULL);
        if (st != OR_OK) {
#ifdef _OPENMP
#pragma omp critical
#endif
          {
            if (status == OR_OK) { status = st; ba = a; bb = b; }
          }
        }
        Mall[(int64_t)a * r + b] = I;
        Mall[(int64_t)b * r + a] = -I;
        if (Ball) Ball[(int64_t)a * r + b] = Ball[(int64_t)b * r + a] = corr;
      }
    }
    free(scratch);
  }
  if (status == OR_OK) {
    for (int32_t a = 0; a < r; ++a) {
      csum s = {0, 0};
      for (int32_t b = 0; b < r; ++b) {
        if (b == a) continue;
        double m = Mall[(int64_t)a * r + b] < 0.0 ? Mall[(int64_t)a * r + b] : 0.0;
        cs_add(&s, m * m);
      }
      S[a] = cs_val(&s);
    }
    if (Mrow) memcpy(Mrow, Mall, sizeof(double) * (size_t)r * (size_t)r);
    if (Brow) memcpy(Brow, Ball, sizeof(double) * (size_t)r * (size_t)r);
  }
  free(Mall); free(Ball);
  if (bad_a) *bad_a = ba;
  if (bad_b) *bad_b = bb;
  return status;
}

/* Normalise every row in U (from the current samples) and take H of each. */
static int normalize_and_entropy(const double* X, double* Z, int64_t n, const int32_t* U,
                                 int32_t r, double* H, int32_t* bad) {
  int status = OR_OK;
  for (int32_t a = 0; a < r; ++a) {
    const double* x = X + (int64_t)U[a] * n;
    double* z = Z + (int64_t)U[a] * n;
    int st = normalize_row(x, n, z, 0.0);
    if (st != OR_OK) { if (bad) *bad = U[a]; return st; }
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int32_t a = 0; a < r; ++a) H[a] = oracle_entropy(Z + (int64_t)U[a] * n, n);
  return status;
}

/* RegressRoot (Alg. 1): x_u <- x_u - cov(x_u, x_root)/var(x_root) x_root
 * for every u remaining in U (root already removed).  Works on the
 * normalised rows Z and writes the residuals back into X. */
static void regress_root(double* X, const double* Z, int64_t n, const int32_t* U, int32_t r,
                         int32_t root) {
  const double* zr = Z + (int64_t)root * n;
  double vr = cov_of(zr, zr, n);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int32_t a = 0; a < r; ++a) {
    const double* zu = Z + (int64_t)U[a] * n;
    double* xu = X + (int64_t)U[a] * n;
    double coef = cov_of(zu, zr, n) / vr;
    for (int64_t k = 0; k < n; ++k) xu[k] = zu[k] - coef * zr[k];
  }
}

/*
 * Full causal-order search (Alg. 1 without its final estimate of B, with Alg. 2).
 *   X         : p x n input, row i = the n samples of variable i (read only)
 *   max_roots : 0 = full order, else stop after this many scored roots
 *   forced    : optional prefix of roots to follow instead of argmax
 *               (scores are still computed and reported)
 *   nthreads  : OpenMP threads, <= 0 = default
 *   order     : [p] out, order[t] = original index of the t-th root;
 *               entries past the last root found are -1
 *   T         : optional [p*p] out, T[t*p + v] = -S_v at iteration t,
 *               NaN if v is not in U at t (or t was not run)
 *   Hout      : optional [p*p] out, Hout[t*p + v] = H(x_v) of the normalised
 *               variable v at iteration t (NaN if not computed)
 *   M         : optional [M_iters*p*p] out, M[t*p*p + i*p + j] = I for the
 *               ordered pair (i, j) at iteration t, NaN where undefined
 *   Bout      : optional [M_iters*p*p] out, correlation of the normalised pair
 *               (i, j) at iteration t (the regression coefficient), NaN where undefined
 *   bad_i/j   : variables of a degenerate or non-finite input
 *   pair_once : evaluate each unordered pair once and take the reverse test as
 *               its negation (bitwise the same outputs, half the work)
 * Returns OR_OK or an error status.
 */
int oracle_fit_order(const double* X, int64_t n, int64_t p, int32_t max_roots,
                     const int32_t* forced, int32_t forced_len, int32_t nthreads,
                     int32_t* order, double* T, double* Hout, double* M, double* Bout,
                     int32_t M_iters, int32_t* bad_i, int32_t* bad_j, int32_t pair_once) {
  if (!X || !order || n < 2 || p < 1) return OR_E_INVALID;
  if (forced_len < 0 || (forced_len > 0 && !forced)) return OR_E_INVALID;
  if (bad_i) *bad_i = -1;
  if (bad_j) *bad_j = -1;
  for (int64_t t = 0; t < p; ++t) order[t] = -1;
  if (T) for (int64_t k = 0; k < p * p; ++k) T[k] = NAN;
  if (Hout) for (int64_t k = 0; k < p * p; ++k) Hout[k] = NAN;
  if (M) for (int64_t k = 0; k < (int64_t)M_iters * p * p; ++k) M[k] = NAN;
  if (Bout) for (int64_t k = 0; k < (int64_t)M_iters * p * p; ++k) Bout[k] = NAN;
  for (int64_t k = 0; k < p * n; ++k)
    if (!isfinite(X[k])) {
      if (bad_i) *bad_i = (int32_t)(k / n);
      return OR_E_NONFINITE;
    }

  size_t pn = (size_t)p * (size_t)n;
  double* W = (double*)malloc(sizeof(double) * pn);  /* current data */
  double* Z = (double*)malloc(sizeof(double) * pn);  /* normalised data */
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * (size_t)p);
  double* H = (double*)malloc(sizeof(double) * (size_t)p);
  double* S = (double*)malloc(sizeof(double) * (size_t)p);
  double* Mr = M ? (double*)malloc(sizeof(double) * (size_t)p * (size_t)p) : NULL;
  double* Br = Bout ? (double*)malloc(sizeof(double) * (size_t)p * (size_t)p) : NULL;
  uint8_t* used = (uint8_t*)calloc((size_t)p, 1);
  if (!W || !Z || !U || !H || !S || !used || (M && !Mr) || (Bout && !Br)) {
    free(W); free(Z); free(U); free(H); free(S); free(Mr); free(Br); free(used);
    return OR_E_NOMEM;
  }
  memcpy(W, X, sizeof(double) * pn);
  int32_t r = (int32_t)p;
  for (int32_t a = 0; a < r; ++a) U[a] = a;  /* U = all variables (Alg. 1) */

  int status = OR_OK;
  int32_t t = 0;
  int32_t limit = max_roots > 0 && max_roots < p ? max_roots : (int32_t)p;
  while (r > 0 && t < limit) {
    int32_t root;
    if (r == 1) {
      /* a single remaining variable is the root (Alg. 2) */
      root = 0;
      if (forced && t < forced_len && forced[t] != U[0]) { status = OR_E_INVALID; break; }
      if (T) T[(int64_t)t * p + U[0]] = 0.0;
    } else {
      int32_t bad = -1;
      status = normalize_and_entropy(W, Z, n, U, r, H, &bad);
      if (status != OR_OK) { if (bad_i) *bad_i = bad; break; }
      int32_t ba = -1, bb = -1;
      const int rec = t < M_iters;
      status = find_root_scores(Z, n, U, r, H, S, rec ? Mr : NULL, rec ? Br : NULL, NULL,
                                nthreads, &ba, &bb, pair_once);
      if (status != OR_OK) {
        if (bad_i) *bad_i = ba >= 0 ? U[ba] : -1;
        if (bad_j) *bad_j = bb >= 0 ? U[bb] : -1;
        break;
      }
      if (T) for (int32_t a = 0; a < r; ++a) T[(int64_t)t * p + U[a]] = -S[a];
      if (Hout) for (int32_t a = 0; a < r; ++a) Hout[(int64_t)t * p + U[a]] = H[a];
      if (M && t < M_iters) {
        for (int32_t a = 0; a < r; ++a)
          for (int32_t b = 0; b < r; ++b)
            M[(int64_t)t * p * p + (int64_t)U[a] * p + U[b]] = Mr[(int64_t)a * r + b];
      }
      if (Bout && t < M_iters) {
        for (int32_t a = 0; a < r; ++a)
          for (int32_t b = 0; b < r; ++b)
            Bout[(int64_t)t * p * p + (int64_t)U[a] * p + U[b]] = Br[(int64_t)a * r + b];
      }
      if (forced && t < forced_len) {
        root = -1;
        for (int32_t a = 0; a < r; ++a) if (U[a] == forced[t]) root = a;
        if (root < 0) { status = OR_E_INVALID; break; }
      } else {
        /* root = argmin S (Alg. 2), first (lowest index) on ties */
        root = 0;
        for (int32_t a = 1; a < r; ++a) if (S[a] < S[root]) root = a;
      }
    }
    int32_t root_var = U[root];
    order[t] = root_var;              /* append the root to K */
    used[root_var] = 1;
    for (int32_t a = root; a + 1 < r; ++a) U[a] = U[a + 1];  /* remove it from U */
    --r;
    ++t;
    if (r > 0 && t < limit) regress_root(W, Z, n, U, r, root_var);  /* RegressRoot */
  }
  free(W); free(Z); free(U); free(H); free(S); free(Mr); free(Br); free(used);
  return status;
}

/*
 * Sampled check at a given iteration, for sizes where the full search is
 * too slow.  Follows the root prefix `prefix[0..t)` (plain RegressRoot after
 * each), then, at iteration t, returns
 *   T_out[k]  = -S_v for v = vars[k]   (k < nvars; needs all r-1 tests of v)
 *   M_out[k]  = I for the ordered pair (pi[k], pj[k])   (k < npairs)
 *   B_out[k]  = correlation of that normalised pair (optional)
 * Variables must still be in U at iteration t.
 */
int oracle_sampled_at(const double* X, int64_t n, int64_t p, const int32_t* prefix, int32_t t,
                      const int32_t* vars, int32_t nvars, double* T_out,
                      const int32_t* pi, const int32_t* pj, int32_t npairs, double* M_out,
                      double* B_out, int32_t nthreads) {
  if (!X || n < 2 || p < 1 || t < 0 || t >= p || (t > 0 && !prefix)) return OR_E_INVALID;
  size_t pn = (size_t)p * (size_t)n;
  double* W = (double*)malloc(sizeof(double) * pn);
  double* Z = (double*)malloc(sizeof(double) * pn);
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * (size_t)p);
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)p);
  double* H = (double*)malloc(sizeof(double) * (size_t)p);
  double* S = (double*)malloc(sizeof(double) * (size_t)p);
  uint8_t* only = (uint8_t*)calloc((size_t)p, 1);
  if (!W || !Z || !U || !pos || !H || !S || !only) {
    free(W); free(Z); free(U); free(pos); free(H); free(S); free(only);
    return OR_E_NOMEM;
  }
  memcpy(W, X, sizeof(double) * pn);
  int32_t r = (int32_t)p;
  for (int32_t a = 0; a < r; ++a) U[a] = a;
  int status = OR_OK;
  for (int32_t s = 0; s < t && status == OR_OK; ++s) {
    status = normalize_and_entropy(W, Z, n, U, r, H, NULL);
    if (status != OR_OK) break;
    int32_t root = -1;
    for (int32_t a = 0; a < r; ++a) if (U[a] == prefix[s]) root = a;
    if (root < 0) { status = OR_E_INVALID; break; }
    int32_t root_var = U[root];
    for (int32_t a = root; a + 1 < r; ++a) U[a] = U[a + 1];
    --r;
    regress_root(W, Z, n, U, r, root_var);
  }
  if (status == OR_OK) status = normalize_and_entropy(W, Z, n, U, r, H, NULL);
  if (status == OR_OK) {
    for (int32_t v = 0; v < p; ++v) pos[v] = -1;
    for (int32_t a = 0; a < r; ++a) pos[U[a]] = a;
    for (int32_t k = 0; k < nvars && status == OR_OK; ++k) {
      if (vars[k] < 0 || vars[k] >= p || pos[vars[k]] < 0) status = OR_E_INVALID;
      else only[pos[vars[k]]] = 1;
    }
    for (int32_t k = 0; k < npairs && status == OR_OK; ++k)
      if (pi[k] < 0 || pi[k] >= p || pj[k] < 0 || pj[k] >= p || pos[pi[k]] < 0 ||
          pos[pj[k]] < 0 || pi[k] == pj[k])
        status = OR_E_INVALID;
  }
  if (status == OR_OK && nvars > 0) {
    status = find_root_scores(Z, n, U, r, H, S, NULL, NULL, only, nthreads, NULL, NULL, 0);
    if (status == OR_OK)
      for (int32_t k = 0; k < nvars; ++k) T_out[k] = -S[pos[vars[k]]];
  }
  if (status == OR_OK && npairs > 0) {
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
      double* scratch = (double*)malloc(sizeof(double) * 2 * (size_t)n);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
      for (int32_t k = 0; k < npairs; ++k) {
        int32_t a = pos[pi[k]], b = pos[pj[k]];
        double I = NAN, corr = NAN;
        if (scratch &&
            compare_normalized(Z + (int64_t)U[a] * n, Z + (int64_t)U[b] * n, H[a], H[b], n,
                               scratch, &I, &corr) != OR_OK)
          I = NAN;
        M_out[k] = I;
        if (B_out) B_out[k] = corr;
      }
      free(scratch);
    }
  }
  free(W); free(Z); free(U); free(pos); free(H); free(S); free(only);
  return status;
}
