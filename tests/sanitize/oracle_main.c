/* Drives the CPU oracle's entry points through searches of several shapes
 * (ordered and pair-once evaluation, forced prefixes, recorded tests),
 * sampled scores, degenerate and non-finite inputs.  Run under ASan/UBSan:
 * any sanitizer report aborts the program; a wrong status or a difference
 * between the two evaluation orders prints and exits 1. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_fit_order(const double* X, int64_t n, int64_t p, int32_t max_roots, const int32_t* forced,
                     int32_t forced_len, int32_t nthreads, int32_t* order, double* T, double* Hout, double* M,
                     double* Bout, int32_t M_iters, int32_t* bad_i, int32_t* bad_j, int32_t pair_once);
int oracle_sampled_at(const double* X, int64_t n, int64_t p, const int32_t* prefix, int32_t t,
                      const int32_t* vars, int32_t nvars, double* T_out, const int32_t* pi, const int32_t* pj,
                      int32_t npairs, double* M_out, double* B_out, int32_t nthreads);
int oracle_compare(const double* xi, const double* xj, int64_t n, double* I_out);
double oracle_entropy(const double* u, int64_t n);
void oracle_entropy_moments(const double* u, int64_t n, double* E1, double* E2);
int oracle_standardize(const double* x, int64_t n, double* z);

static int fail = 0;
static uint64_t rs = 88172645463325252ull;
static double urand(void) {
  rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
  return (double)(rs >> 11) * 0x1.0p-53 - 0.5;
}

static void check(int cond, const char* what) {
  if (!cond) { printf("FAIL %s\n", what); fail = 1; }
}

static int same(const double* a, const double* b, size_t k) {
  for (size_t i = 0; i < k; ++i)
    if (!(a[i] == b[i] || (isnan(a[i]) && isnan(b[i])))) return 0;
  return 1;
}

static void search(int64_t p, int64_t n, int threads) {
  double* X = malloc(sizeof(double) * p * n);
  for (int64_t k = 0; k < p * n; ++k) X[k] = urand();
  /* a chain so the search has structure */
  for (int64_t i = 1; i < p; ++i)
    for (int64_t k = 0; k < n; ++k) X[i * n + k] += 0.7 * X[(i - 1) * n + k];
  const int32_t rec = p < 3 ? (int32_t)p : 3;
  int32_t *o1 = malloc(4 * p), *o2 = malloc(4 * p), bi, bj;
  double *T1 = malloc(8 * p * p), *T2 = malloc(8 * p * p), *H1 = malloc(8 * p * p), *H2 = malloc(8 * p * p);
  double *M1 = malloc(8 * rec * p * p), *M2 = malloc(8 * rec * p * p);
  double *B1 = malloc(8 * rec * p * p), *B2 = malloc(8 * rec * p * p);
  check(oracle_fit_order(X, n, p, 0, NULL, 0, threads, o1, T1, H1, M1, B1, rec, &bi, &bj, 0) == 0, "ordered search");
  check(oracle_fit_order(X, n, p, 0, NULL, 0, threads, o2, T2, H2, M2, B2, rec, &bi, &bj, 1) == 0, "pair-once search");
  check(memcmp(o1, o2, 4 * p) == 0, "orders of the two evaluations");
  check(same(T1, T2, p * p) && same(H1, H2, p * p) && same(M1, M2, rec * p * p), "scores of the two evaluations");
  /* forced prefix and max_roots */
  if (p >= 3) {
    int32_t pre[2] = {(int32_t)(p - 1), 0};
    check(oracle_fit_order(X, n, p, 2, pre, 2, threads, o2, T2, NULL, NULL, NULL, 0, &bi, &bj, 1) == 0, "forced");
    check(o2[0] == p - 1 && o2[1] == 0 && o2[2] == -1, "forced prefix followed");
    /* sampled scores at iteration 1 after the same prefix */
    int32_t vars[2] = {1, (int32_t)(p - 2)}, pi[2] = {1, 2}, pj[2] = {2, 1};
    double Ts[2], Ms[2], Bs[2];
    check(oracle_sampled_at(X, n, p, pre, 1, vars, 2, Ts, pi, pj, 2, Ms, Bs, threads) == 0, "sampled_at");
    check(Ms[0] == -Ms[1], "sampled antisymmetry");
    check(oracle_sampled_at(X, n, p, pre, (int32_t)p, vars, 2, Ts, pi, pj, 2, Ms, Bs, threads) != 0,
          "sampled_at t out of range");
  }
  free(X); free(o1); free(o2); free(T1); free(T2); free(H1); free(H2); free(M1); free(M2); free(B1); free(B2);
}

int main(void) {
  search(1, 16, 1);
  search(2, 5, 1);
  search(9, 700, 2);
  search(17, 257, 4);
  search(30, 1000, 8);

  /* pair, entropy and normalisation entry points */
  {
    const int64_t n = 513;
    double *a = malloc(8 * n), *b = malloc(8 * n), *z = malloc(8 * n), I, E1, E2;
    for (int64_t k = 0; k < n; ++k) { a[k] = urand(); b[k] = urand() + 0.5 * a[k]; }
    check(oracle_compare(a, b, n, &I) == 0 && isfinite(I), "compare");
    check(oracle_standardize(a, n, z) == 0, "standardize");
    check(isfinite(oracle_entropy(z, n)), "entropy");
    oracle_entropy_moments(z, n, &E1, &E2);
    check(isfinite(E1) && isfinite(E2), "moments");
    for (int64_t k = 0; k < n; ++k) b[k] = 3.0 * a[k] + 1.0;   /* exactly collinear */
    check(oracle_compare(a, b, n, &I) != 0, "collinear pair is degenerate");
    free(a); free(b); free(z);
  }

  /* degenerate and non-finite inputs, argument errors */
  {
    const int64_t p = 6, n = 300;
    double* X = malloc(8 * p * n);
    int32_t order[6], bi, bj;
    for (int64_t k = 0; k < p * n; ++k) X[k] = urand();
    for (int64_t k = 0; k < n; ++k) X[3 * n + k] = 2.0;           /* zero variance */
    check(oracle_fit_order(X, n, p, 0, NULL, 0, 2, order, NULL, NULL, NULL, NULL, 0, &bi, &bj, 1) == 3 && bi == 3,
          "zero-variance row");
    for (int64_t k = 0; k < n; ++k) X[3 * n + k] = -X[k];         /* collinear with row 0 */
    check(oracle_fit_order(X, n, p, 0, NULL, 0, 2, order, NULL, NULL, NULL, NULL, 0, &bi, &bj, 0) == 3,
          "collinear rows");
    X[3 * n + 5] = NAN;
    check(oracle_fit_order(X, n, p, 0, NULL, 0, 2, order, NULL, NULL, NULL, NULL, 0, &bi, &bj, 1) == 2 && bi == 3,
          "non-finite sample");
    check(oracle_fit_order(NULL, n, p, 0, NULL, 0, 2, order, NULL, NULL, NULL, NULL, 0, &bi, &bj, 1) == 1, "null X");
    check(oracle_fit_order(X, 1, p, 0, NULL, 0, 2, order, NULL, NULL, NULL, NULL, 0, &bi, &bj, 1) == 1, "n = 1");
    for (int64_t k = 0; k < n; ++k) X[3 * n + k] = urand();
    int32_t dup[2] = {1, 1};
    check(oracle_fit_order(X, n, p, 0, dup, 2, 2, order, NULL, NULL, NULL, NULL, 0, &bi, &bj, 1) == 1,
          "duplicate forced root");
    free(X);
  }
  printf(fail ? "oracle host checks FAILED\n" : "oracle host checks passed\n");
  return fail;
}
