// HIP kernels (gfx950) of the DirectLiNGAM causal-order search.
//
// Paper: Shahbazinia, Salehkaleybar, Hashemi, "ParaLiNGAM: Parallel Causal
// Structure Learning for Linear non-Gaussian Acyclic Models", arXiv 2109.13993.
//
//   k_standardize  NormalizeData (Alg. 3, first Par step): row mean and
//                  adjusted (n-1) variance in binary64, z = (x - mean)/sd.
//   k_gram         CalculateCovMat (Alg. 3): Sigma = Z Z^T / (n-1) with the
//                  binary64 matrix cores (v_mfma_f64_16x16x4f64); also the
//                  refresh of Sigma after each UpdateData.
//   k_entropy      H(x_u) of Eq. (HApp) for every remaining variable (the two
//                  per-variable terms of Eq. (Itest), computed once per
//                  iteration), and the iteration's set-up.
//   k_pair_band    Compare for a band of pair tiles (Alg. 2 body, Eq. (Itest),
//                  Eq. (HApp)): the residuals r_i^(j) and r_j^(i), normalised by
//                  1/sqrt(1 - b^2) (Eq. var_update), are formed on the fly from two
//                  rows staged through LDS and reduced over samples; each
//                  unordered pair is evaluated once (messaging, Sec. 3.1) and only
//                  if one of its variables is below the threshold (Sec. 3.2).
//   k_score        Forms I for the evaluated pairs, the scores
//                  S_i = sum_j min(0, I_ij)^2 and the threshold state; its last
//                  work-group applies the termination test and the threshold
//                  update of the Scheduler (Alg. 6 / Sec. 4.3) and picks the root.
//   k_rank         Positions of the survivors for the next iteration, in order
//                  of their score in this one.
//   k_update_*     UpdateData and UpdateCovMat (Sec. 3.4): rank-1 update of the
//                  remaining rows and of Sigma into their new positions (the
//                  row update also sums the next iteration's entropy terms
//                  when no Gram refresh follows); the iteration's results are
//                  recorded first.
#include "lingam_internal.h"
#include "fp64_math.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>

#include <cmath>
#include <type_traits>

namespace lingam {

// Kernel arguments naming the data sets of a launch: a batch of one passes
// its descriptor by value (no extra dependent load before a kernel can find
// its buffers); a larger batch passes the device array.
#define DEVS(b) ((b).count == 1 ? nullptr : (b).dd), (b).one

namespace {

// Eq. (HApp) constants as printed; H(nu) = (1 + log 2 pi) / 2.
constexpr double K1 = 79.047;
constexpr double K2 = 7.4129;
constexpr double BETA = 0.37457;
constexpr double HNU = 1.4189385332046727418;
constexpr double LN2 = 0.69314718055994530942;
constexpr float LOG2E_F = 1.44269504088896340736f;

// Variables left in data set d at iteration t (0 once its iterations are done).
__device__ __forceinline__ int rows_left(const Dev& d, int t) { return t < d.limit ? d.p - t : 0; }

__device__ __forceinline__ bool halted(const Ctl* c) {
  return __atomic_load_n(&c->halt, __ATOMIC_RELAXED) != 0;
}

__device__ void raise_error(Ctl* c, int32_t st, int32_t bi, int32_t bj) {
  if (atomicCAS(&c->status, ST_OK, st) == ST_OK) {
    c->bad_i = bi;
    c->bad_j = bj;
  }
  atomicExch(&c->halt, 1);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// Sum over a work-group of 256 threads in a fixed order; result to all threads.
__device__ double block_sum256(double x, double* sh) {
  x = wave_sum(x);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = x;
  __syncthreads();
  double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

__device__ int block_or256(int x, int* sh) {
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  int any = __any(x) ? 1 : 0;
  __syncthreads();
  if (l == 0) sh[w] = any;
  __syncthreads();
  int t = sh[0] | sh[1] | sh[2] | sh[3];
  __syncthreads();
  return t;
}

// ---- element terms of Eq. (HApp) ------------------------------------------
// FP64: log cosh(u) + log 2 = |u| + log1p(exp(-2|u|)); g(u) = u exp(-u^2/2).
// The logarithm's argument lies in [0, 1], the range of log1p_unit.
__device__ __forceinline__ void terms_f64(double u, double& lc, double& g) {
  const double a = fabs(u);
  lc += a + log1p_unit(exp(-2.0 * a));
  g += u * exp(-0.5 * u * u);
}

// Mixed: u = s * x with x the unscaled residual in binary32.  With
// ca = -2 log2(e) s and cg = -log2(e) s^2 / 2:
//   a2 = ca |x| = -2 log2(e) |u|,  log2(1 + 2^a2) - a2/2 = (log cosh u + ln 2)/ln 2,
//   2^(cg x^2) = exp(-u^2 / 2),   x 2^(cg x^2) = g(u) / s.
__device__ __forceinline__ void terms_mixed(float x, float ca, float cg, float& lc, float& g) {
  const float a2 = fabsf(x) * ca;
  const float e1 = __builtin_amdgcn_exp2f(a2);
  const float l = __builtin_amdgcn_logf(1.0f + e1);
  lc += __builtin_fmaf(a2, -0.5f, l);
  const float t = x * cg;
  const float e2 = __builtin_amdgcn_exp2f(t * x);
  g = __builtin_fmaf(x, e2, g);
}

// Rounding bounds of one entropy estimate of the mixed modes, from its sums
// s_lc = sum (log cosh u + ln 2) and s_g = sum u exp(-u^2/2) over n samples
// of a unit-variance u (so mean |u| <= 1 and mean u^2 = 1).  u32 = 2^-24;
// the hardware exp2 and log2 are within E = LINGAM_EXP2_ERR u32 (relative)
// and L = LINGAM_LOG2_ERR u32 (absolute) on the arguments used, which
// lingam_check_terms measures.  Per term t of log cosh (natural units):
// the argument of exp2 carries 3 u32 (residual, scale and product
// roundings), which the final fma halves: 3.0 u32 |u|; exp2, the add and
// log2: (2.10 + E + ln 2 L) u32; the fma u32 |t|.  Per term of
// g = u exp(-u^2/2): 5 u32 on the exp2 argument gives 2.5 u32 |u|^3 e^-u^2/2
// <= 2.9 u32, exp2 and the operand (1 + E) u32 |g|, the fma u32 |g|, with
// |g| <= e^-1/2.  Lane sums of at most 32 terms in binary32.
//
// Worst case (happ_err_mixed): every error at its bound, lane sums at
// 31 u32 sum |t|:
//   dE1 <= u32 (32 s_lc / n + 3.0 + 2.10 + E + ln 2 L),
//   dE2 <= u32 (32 e^-1/2 + (1 + E) e^-1/2 + 2.9).
// Probable (happ_err_prob): the rounding errors of round-to-nearest
// operations and the hardware functions' deviations from their mean are
// modelled as independent, zero-mean and bounded by the same amounts;
// Hoeffding's inequality then bounds their sum by lambda times the root of
// the sum of the squared bounds with probability at least
// 1 - 2 exp(-lambda^2 / 2) (lambda = 8: 2.5e-14 per estimate).  The lane
// sums' roundings u32 S_j (S_j a partial sum) have sum of squares at most
// 1024 sum t^2 (S_j <= S_32, S_32^2 <= 32 sum t^2 over the lane) and
// 528 sum g^2 for the signed g terms; with mean t^2 <= 2 + 2 ln^2 2 and
// g^2 <= 1/e this gives
//   dE1 <= u32 (ln 2 bL + bE + 8 sqrt(3158 / n)),
//   dE2 <= u32 (e^-1/2 bE + 8 sqrt(223 / n)),
// where bE = LINGAM_EXP2_BIAS and bL = LINGAM_LOG2_BIAS bound the hardware
// functions' systematic error (the largest mean error within a binade,
// measured by lingam_check_terms) and stay additive.
// Eq. (HApp) then moves by at most
//   2 k1 |E1 - beta| dE1 + 3 k1 dE1^2 + 2 k2 |E2| dE2 + 3 k2 dE2^2
// (E1, E2 the computed means; the factor 3 absorbs using them in place of the
// exact ones).
//
// s_in (FP32 storage only, else 0) is the residual's scale 1/sqrt(1 - b^2):
// a residual u = s (z_v - b z_w) formed by one binary32 fma from rows stored
// to u32 and b rounded to binary32 moves by at most u32 s (|z_v| + 2 |z_w|)
// beyond its own rounding; both term derivatives are at most 1 in magnitude
// and mean |z| <= 1, so each moment moves by at most 3 s u32 more in the
// worst case.  In the probable bound the rounding of b is one error shared
// by all samples (s u32, additive) and the storage and fma roundings are
// per-sample (3 s u32 each, under the square root).
constexpr double U32 = 5.9604644775390625e-08;
constexpr double HOEFFDING_LAMBDA = 8.0;

__device__ __forceinline__ double happ_move(double E1, double E2, double d1, double d2) {
  return 2.0 * K1 * fabs(E1 - BETA) * d1 + 3.0 * K1 * d1 * d1 + 2.0 * K2 * fabs(E2) * d2 + 3.0 * K2 * d2 * d2;
}

__device__ __forceinline__ double happ_err_mixed(double s_lc, double s_g, double n, double s_in = 0.0) {
  constexpr double E = LINGAM_EXP2_ERR, L = LINGAM_LOG2_ERR, G = 0.60653065971263342;  // e^-1/2
  const double d1 = U32 * (32.0 * (s_lc / n) + 3.0 + 2.10 + E + LN2 * L + 3.0 * s_in);
  const double d2 = U32 * (32.0 * G + (1.0 + E) * G + 2.9 + 3.0 * s_in);
  return happ_move(s_lc / n - LN2, s_g / n, d1, d2);
}

__device__ __forceinline__ double happ_err_prob(double s_lc, double s_g, double n, double s_in = 0.0) {
  constexpr double bE = LINGAM_EXP2_BIAS, bL = LINGAM_LOG2_BIAS, G = 0.60653065971263342;
  const double r1 = 3158.0 + 9.0 * s_in * s_in, r2 = 223.0 + 9.0 * s_in * s_in;
  const double d1 = U32 * (LN2 * bL + bE + s_in + HOEFFDING_LAMBDA * sqrt(r1 / n));
  const double d2 = U32 * (G * bE + s_in + HOEFFDING_LAMBDA * sqrt(r2 / n));
  return happ_move(s_lc / n - LN2, s_g / n, d1, d2);
}

__device__ __forceinline__ double happ_from_sums(double s_lc, double s_g, double n) {
  // s_lc = sum (log cosh u + ln 2), s_g = sum u exp(-u^2/2)
  const double E1 = s_lc / n - LN2;
  const double E2 = s_g / n;
  const double d1 = E1 - BETA;
  return HNU - K1 * d1 * d1 - K2 * E2 * E2;
}

}  // namespace

// ============================================================================
// a1: NormalizeData
// ============================================================================
template <typename T, int LAYOUT, typename S>
__device__ void standardize_row(const T* __restrict__ X, int64_t n, int p, int i, S* __restrict__ Z,
                                int64_t ldz, Ctl* ctl, double* stats) {
  __shared__ double sh[4];
  __shared__ int shi[4];
  auto load = [&](int64_t k) -> double {
    return LAYOUT == 0 ? (double)X[(int64_t)i * n + k] : (double)X[k * (int64_t)p + i];
  };
  double s = 0.0, sc = 0.0;  // Kahan sum of the samples of this thread
  int bad = 0;
  for (int64_t k = threadIdx.x; k < n; k += 256) {
    const double x = load(k);
    if (!isfinite(x)) bad = 1;
    const double y = x - sc, t = s + y;
    sc = (t - s) - y;
    s = t;
  }
  if (block_or256(bad, shi)) {
    if (threadIdx.x == 0) raise_error(ctl, ST_NONFINITE, i, -1);
    return;
  }
  const double mean = block_sum256(s, sh) / (double)n;
  double q = 0.0, qc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) {
    const double dx = load(k) - mean;
    const double y = dx * dx - qc, t = q + y;
    qc = (t - q) - y;
    q = t;
  }
  const double var = block_sum256(q, sh) / (double)(n - 1);
  if (!(var > 0.0) || !isfinite(var)) {
    if (threadIdx.x == 0) raise_error(ctl, isfinite(var) ? ST_DEGENERATE : ST_NONFINITE, i, -1);
    return;
  }
  const double sd = sqrt(var);
  S* z = Z + (int64_t)i * ldz;
  for (int64_t k = threadIdx.x; k < ldz; k += 256) z[k] = k < n ? (S)((load(k) - mean) / sd) : (S)0;
  if (threadIdx.x == 0 && stats) {
    stats[2 * i] = mean;
    stats[2 * i + 1] = var;
  }
}

// One work-group per row (blockIdx.x) of data set blockIdx.z.
template <typename S>
__device__ __forceinline__ void standardize_into(const Dev& d, int i) {
  S* Z = static_cast<S*>(d.Z[0]);
  if (d.x_dtype == 0 && d.layout == 0)
    standardize_row<double, 0, S>((const double*)d.X, d.n, d.p, i, Z, d.ldz, d.ctl, d.stats);
  else if (d.x_dtype == 0)
    standardize_row<double, 1, S>((const double*)d.X, d.n, d.p, i, Z, d.ldz, d.ctl, d.stats);
  else if (d.layout == 0)
    standardize_row<float, 0, S>((const float*)d.X, d.n, d.p, i, Z, d.ldz, d.ctl, d.stats);
  else
    standardize_row<float, 1, S>((const float*)d.X, d.n, d.p, i, Z, d.ldz, d.ctl, d.stats);
}

__device__ __forceinline__ void k_standardize_body(const Dev& d) {
  const int i = blockIdx.x;
  if (i >= d.p) return;
  if (d.store32)
    standardize_into<float>(d, i);
  else
    standardize_into<double>(d, i);
}

__global__ __launch_bounds__(256) void k_standardize(const Dev* __restrict__ devs, const Dev one) {
  if (devs)
    k_standardize_body(devs[blockIdx.z]);
  else
    k_standardize_body(one);
}

hipError_t launch_standardize(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_standardize, dim3(b.p_max, 1, b.count), dim3(256), 0, s, DEVS(b));
  return hipGetLastError();
}

// Bootstrap resample: out[i][k] = X[i][idx[k]] for the p rows of a p x n_src
// binary64 matrix (row = variable).
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ X, int64_t n_src,
                                                const int64_t* __restrict__ idx, int64_t n_idx,
                                                double* __restrict__ out) {
  const int i = blockIdx.y;
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n_idx; k += (int64_t)gridDim.x * 256) {
    const int64_t j = idx[k];
    out[(int64_t)i * n_idx + k] = (j >= 0 && j < n_src) ? X[(int64_t)i * n_src + j] : __builtin_nan("");
  }
}

hipError_t launch_gather(const double* X, int64_t n_src, int64_t p, const int64_t* idx, int64_t n_idx,
                         double* out, hipStream_t s) {
  const int xb = (int)std::min<int64_t>(64, (n_idx + 255) / 256);
  hipLaunchKernelGGL(k_gather, dim3(std::max(xb, 1), (unsigned)p), dim3(256), 0, s, X, n_src, idx, n_idx, out);
  return hipGetLastError();
}

// ============================================================================
// a2: CalculateCovMat / refresh -- Sigma = Z Z^T / (n-1) on the FP64 matrix cores
// ============================================================================
typedef double dbl4 __attribute__((ext_vector_type(4)));
// Partial Gram of one sample slice: Gp[slice][i][j] = sum_{k in slice} z_i[k] z_j[k]
// (slice stride r rows of p: the buffer holds the most slices times rows any r needs)
// for the upper-triangular 32 x 32 tile given by blockIdx.x (i <= j).  Each
// LDS stage is summed by the matrix cores into a fresh accumulator and then
// added into a Kahan-compensated total; the next stage is fetched into
// registers while the current one is multiplied.
// Grid: (tiles, slices, data sets), sized for the largest data set; each
// data set uses its own tile and slice counts (the same as when it runs
// alone), and the surplus work-groups return.
template <typename S>
__device__ __forceinline__ void k_gram_partial_body(const Dev& d, int buf, int t) {
  const int r = rows_left(d, t);
  if (r < 1 || halted(d.ctl)) return;
  const S* __restrict__ Z = static_cast<const S*>(d.Z[buf]);
  const int64_t ldz = d.ldz, n = d.n;
  double* __restrict__ Gp = d.Gp;
  const int ldg = d.p;
  const int nsl = gram_slices(r, n, d.gram_slices_max);  // this data set's own split
  if ((int)blockIdx.y >= nsl) return;
  const int64_t stages = (n + GK - 1) / GK;
  const int64_t slice_len = (stages + nsl - 1) / nsl * GK;
  __shared__ double As[GT][GK + 1];
  __shared__ double Bs[GT][GK + 1];
  const int nt = (r + GT - 1) / GT;
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int ti = 0, rem = blockIdx.x;
  while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
  const int tj = ti + rem;
  const int i0 = ti * GT, j0 = tj * GT;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wy = wave >> 1, wx = wave & 1;
  const int64_t kbeg = (int64_t)blockIdx.y * slice_len;
  const int64_t kend = min((int64_t)((n + GK - 1) / GK * GK), kbeg + slice_len);  // <= ldz
  // this thread's 8 + 8 elements of a stage
  constexpr int PER = (GT * GK) / 256;
  const int row0 = threadIdx.x / (GK / PER), col0 = (threadIdx.x % (GK / PER)) * PER;
  const bool ra = i0 + row0 < r, rb = j0 + row0 < r;
  const S* za = Z + (int64_t)(i0 + row0) * ldz + col0;
  const S* zb = Z + (int64_t)(j0 + row0) * ldz + col0;
  double pa[PER], pb[PER];
  // binary32 rows are widened exactly, so the Gram is the same binary64
  // contraction of the stored values
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < PER; e += 2) {
      if constexpr (sizeof(S) == 8) {
        double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
        if (ra) va = *reinterpret_cast<const double2*>(za + k0 + e);
        if (rb) vb = *reinterpret_cast<const double2*>(zb + k0 + e);
        pa[e] = va.x; pa[e + 1] = va.y;
        pb[e] = vb.x; pb[e + 1] = vb.y;
      } else {
        float2 va = make_float2(0.f, 0.f), vb = make_float2(0.f, 0.f);
        if (ra) va = *reinterpret_cast<const float2*>(za + k0 + e);
        if (rb) vb = *reinterpret_cast<const float2*>(zb + k0 + e);
        pa[e] = (double)va.x; pa[e + 1] = (double)va.y;
        pb[e] = (double)vb.x; pb[e + 1] = (double)vb.y;
      }
    }
  };
  dbl4 tot = {0.0, 0.0, 0.0, 0.0}, comp = {0.0, 0.0, 0.0, 0.0};
  if (kbeg < kend) fetch(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += GK) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      As[row0][col0 + e] = pa[e];
      Bs[row0][col0 + e] = pb[e];
    }
    __syncthreads();
    if (k0 + GK < kend) fetch(k0 + GK);
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const double a = As[wy * 16 + (lane & 15)][kk + (lane >> 4)];
      const double b = Bs[wx * 16 + (lane & 15)][kk + (lane >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double y = acc[v] - comp[v];
      const double t = tot[v] + y;
      comp[v] = (t - tot[v]) - y;
      tot[v] = t;
    }
    __syncthreads();
  }
  // result layout of v_mfma_f64_16x16x4f64: lane holds rows lane/16 + 4v, column lane%16
  double* G = Gp + (int64_t)blockIdx.y * r * ldg;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gi = i0 + wy * 16 + (lane >> 4) + 4 * v;
    const int gj = j0 + wx * 16 + (lane & 15);
    if (gi < r && gj < r && gi <= gj) G[(int64_t)gi * ldg + gj] = tot[v];
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_gram_partial(const Dev* __restrict__ devs, const Dev one, int buf, int t) {
  if (devs)
    k_gram_partial_body<S>(devs[blockIdx.z], buf, t);
  else
    k_gram_partial_body<S>(one, buf, t);
}

// Sum the slices in a fixed order, scale by 1/(n-1), mirror, and set the row
// scales d_i = 1/sqrt(G_ii).
__device__ __forceinline__ void k_gram_reduce_body(const Dev& d, int buf, int t) {
  const int r = rows_left(d, t);
  if (r < 1 || halted(d.ctl)) return;
  const int nslice = gram_slices(r, d.n, d.gram_slices_max);
  const double* __restrict__ Gp = d.Gp;
  double* __restrict__ Sig = d.Sig[buf];
  double* __restrict__ dsc = d.dsc[buf];
  const int ldg = d.p;
  const double n = (double)d.n;
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (i >= r || j < i || j >= r) return;
  double sum = 0.0;
  for (int q = 0; q < nslice; ++q) sum += Gp[((int64_t)q * r + i) * ldg + j];
  const double val = sum / (n - 1.0);
  Sig[(int64_t)i * ldg + j] = val;
  Sig[(int64_t)j * ldg + i] = val;
  if (i == j) dsc[i] = 1.0 / sqrt(val);
}

__global__ __launch_bounds__(256) void k_gram_reduce(const Dev* __restrict__ devs, const Dev one, int buf, int t) {
  if (devs)
    k_gram_reduce_body(devs[blockIdx.z], buf, t);
  else
    k_gram_reduce_body(one, buf, t);
}

// Gram of the r = p - t rows of buffer buf of every data set.
hipError_t launch_gram(const Batch& b, int buf, int t, hipStream_t s) {
  const int r = b.p_max - t;
  if (r < 1) return hipSuccess;
  const int nt = (r + GT - 1) / GT;
  const dim3 grid(nt * (nt + 1) / 2, b.gram_slices_max, b.count);
  if (b.store32)
    hipLaunchKernelGGL(k_gram_partial<float>, grid, dim3(256), 0, s, DEVS(b), buf, t);
  else
    hipLaunchKernelGGL(k_gram_partial<double>, grid, dim3(256), 0, s, DEVS(b), buf, t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3((r + 255) / 256, r, b.count), dim3(256), 0, s, DEVS(b), buf, t);
  return hipGetLastError();
}

// ============================================================================
// iteration set-up: M = "not evaluated", S = 0, everyone below the threshold
// ============================================================================
// Row x's share, done by the work-group that also forms the row's entropy:
// its tests (row x of M and of the pending flags), its score and threshold
// state; the group of row 0 also sets the iteration's control fields.
// gamma0 > 0: that initial threshold in every iteration; gamma0 <= 0:
// adaptive, `adapt` times the previous iteration's root score (the first
// iteration and a zero previous score use 1e-6).
__device__ __forceinline__ void iter_init_row(const Dev& d, int t, int x, double gamma0, double adapt,
                                              int threshold) {
  const int r = rows_left(d, t), p = d.p;
  Ctl* ctl = d.ctl;
  double* M = d.M + (int64_t)x * p;
  uint8_t* pend = d.pend + (int64_t)x * p;
  for (int w = threadIdx.x; w < r; w += blockDim.x) {
    M[w] = __builtin_nan("");
    pend[w] = 0;
  }
  if (threadIdx.x == 0) {
    d.S[x] = 0.0;
    d.alive[x] = 1;
    d.complete[x] = 0;
    d.alive_list[x] = x;
  }
  // Degeneracy of every pair of the row, pruned or not: a normalised
  // residual needs 1 - b^2 > 0 (Eq. var_update), and the row update divides
  // by sqrt(1 - b^2) for whichever variable becomes the root.  b is formed
  // exactly as the pair kernel forms it.
  {
    const int buf = t & 1;
    const double* sig = d.Sig[buf] + (int64_t)x * p;
    const double* dsc = d.dsc[buf];
    const double dx = dsc[x];
    int bad = -1;
    for (int w = threadIdx.x; w < r; w += blockDim.x) {
      if (w == x) continue;
      const double b = sig[w] * (dx * dsc[w]);
      if (!(1.0 - b * b > DEGEN_EPS)) bad = w;
    }
    if (bad >= 0) {
      const int32_t* idx = d.idx[buf];
      raise_error(ctl, ST_DEGENERATE, idx[x], idx[bad]);
    }
  }
  if (x == 0 && threadIdx.x == 0) {
    double g = gamma0;
    if (!(g > 0.0)) {
      const double prev = ctl->last_root_S;
      g = prev > 0.0 ? adapt * prev : 1e-6;
    }
    ctl->gamma = g;
    ctl->done = 0;
    ctl->root = -1;
    ctl->round = 0;
    ctl->n_alive = r;
    const int nb = (r + TB - 1) / TB;
    ctl->tb_next = 0;
    ctl->ntb_next = threshold ? min(d.band_k0, nb) : nb;
    ctl->iter_bands = 0;
    ctl->arrivals = 0;
    ctl->q_next = 0;
  }
}

// ============================================================================
// a3: per-variable entropy H(x_u), Eq. (HApp)
// ============================================================================
// Sum over a work-group of NT threads in a fixed order; result to all threads.
template <int NT>
__device__ double block_sum(double x, double* sh) {
  constexpr int NW = NT / 64;
  x = wave_sum(x);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// One work-group per row.  A row of n >= ENT_WIDE_N samples is spread over
// W = 1024 threads, a shorter one over W = 256: thread tid takes the samples
// k = tid + W i (binary32 sums of at most 32 of them in the mixed mode), then
// a fixed-order reduction.  W depends only on the data set's own n (threads
// beyond W add exact zeros), so a data set gets the same bits in any launch
// width, alone or in a batch.
constexpr int64_t ENT_WIDE_N = 8192;

// Sample segments of a row of n samples in the row update: at most
// ENT_SEGS, and about 1024 samples or more each (4 per thread), so that
// short rows do not spread over many nearly empty work-groups.
__host__ __device__ inline int entropy_segments_of(int64_t n) {
  const int64_t s = (n + 1023) / 1024;
  return (int)(s < 1 ? 1 : (s < ENT_SEGS ? s : ENT_SEGS));
}

template <bool MIXED, int NT, typename S>
__device__ __forceinline__ void k_entropy_body(const Dev& d, int t, double gamma0, double adapt, int threshold,
                                               int fused) {
  const int r = rows_left(d, t);
  if ((int)blockIdx.x >= r || r < 2 || halted(d.ctl)) return;
  iter_init_row(d, t, (int)blockIdx.x, gamma0, adapt, threshold);
  const int64_t n = d.n;
  double* __restrict__ H = d.H;
  double* __restrict__ eH = d.eH;
  if (fused) {
    // the row update summed the terms per segment: add them up in order
    if (threadIdx.x == 0) {
      const double* hp = d.Hp + (int64_t)blockIdx.x * ENT_SEGS * 2;
      const int segs = entropy_segments_of(n);
      double lc = 0.0, g = 0.0;
      for (int q = 0; q < segs; ++q) {
        lc += hp[2 * q];
        g += hp[2 * q + 1];
      }
      H[blockIdx.x] = happ_from_sums(lc, g, (double)n);
      eH[blockIdx.x] = MIXED ? happ_err_mixed(lc, g, (double)n) : 0.0;
      d.eHp[blockIdx.x] = MIXED ? happ_err_prob(lc, g, (double)n) : 0.0;
    }
    return;
  }
  const int buf = t & 1;
  __shared__ double sh[NT / 64];
  // the row is normalised here, once per iteration: d z is used for the
  // entropy and, when the Gram refresh gave d != 1, stored back in place for
  // the rest of the iteration
  S* z = static_cast<S*>(d.Z[buf]) + (int64_t)blockIdx.x * d.ldz;
  const double dz = d.dsc[buf][blockIdx.x];
  const bool store = dz != 1.0;
  const int W = NT >= 1024 && n >= ENT_WIDE_N ? 1024 : 256;
  double lc = 0.0, g = 0.0;
  if ((int)threadIdx.x < W) {
    if constexpr (MIXED) {
      const float ca = -2.0f * LOG2E_F, cg = -0.5f * LOG2E_F;
      int64_t k = threadIdx.x;
      while (k < n) {
        float flc = 0.f, fg = 0.f;
#pragma unroll 4
        for (int c = 0; c < 32; ++c, k += W)
          if (k < n) {
            // the terms see exactly the value the row then holds
            const double zk = dz * (double)z[k];
            if (store) z[k] = (S)zk;
            terms_mixed((float)zk, ca, cg, flc, fg);
          }
        lc += (double)flc * LN2;
        g += (double)fg;
      }
    } else {
#pragma unroll 4
      for (int64_t k = threadIdx.x; k < n; k += W) {
        const double zk = dz * (double)z[k];
        if (store) z[k] = (S)zk;
        terms_f64(zk, lc, g);
      }
    }
  }
  lc = block_sum<NT>(lc, sh);
  g = block_sum<NT>(g, sh);
  if (threadIdx.x == 0) {
    H[blockIdx.x] = happ_from_sums(lc, g, (double)n);
    eH[blockIdx.x] = MIXED ? happ_err_mixed(lc, g, (double)n) : 0.0;
    d.eHp[blockIdx.x] = MIXED ? happ_err_prob(lc, g, (double)n) : 0.0;
  }
}

template <bool MIXED, int NT, typename S>
__global__ __launch_bounds__(NT) void k_entropy(const Dev* __restrict__ devs, const Dev one, int t, double gamma0,
                                                double adapt, int threshold, int fused) {
  if (devs)
    k_entropy_body<MIXED, NT, S>(devs[blockIdx.z], t, gamma0, adapt, threshold, fused);
  else
    k_entropy_body<MIXED, NT, S>(one, t, gamma0, adapt, threshold, fused);
}

hipError_t launch_iter_start(const Batch& b, int t, double gamma0, double adapt, int threshold, int fused,
                             hipStream_t s) {
  const int r = b.p_max - t;
  if (r < 2) return hipSuccess;
  const dim3 g(r, 1, b.count);
  const bool wide = b.n_max >= ENT_WIDE_N;
  if (b.store32 && wide)
    hipLaunchKernelGGL((k_entropy<true, 1024, float>), g, dim3(1024), 0, s, DEVS(b), t, gamma0, adapt, threshold,
                       fused);
  else if (b.store32)
    hipLaunchKernelGGL((k_entropy<true, 256, float>), g, dim3(256), 0, s, DEVS(b), t, gamma0, adapt, threshold,
                       fused);
  else if (b.mixed && wide)
    hipLaunchKernelGGL((k_entropy<true, 1024, double>), g, dim3(1024), 0, s, DEVS(b), t, gamma0, adapt, threshold,
                       fused);
  else if (b.mixed)
    hipLaunchKernelGGL((k_entropy<true, 256, double>), g, dim3(256), 0, s, DEVS(b), t, gamma0, adapt, threshold,
                       fused);
  else if (wide)
    hipLaunchKernelGGL((k_entropy<false, 1024, double>), g, dim3(1024), 0, s, DEVS(b), t, gamma0, adapt,
                       threshold, fused);
  else
    hipLaunchKernelGGL((k_entropy<false, 256, double>), g, dim3(256), 0, s, DEVS(b), t, gamma0, adapt, threshold,
                       fused);
  return hipGetLastError();
}

// ============================================================================
// a4/a5: the pair kernel
// ============================================================================
// Work of one band: every variable below the threshold ("alive", compacted
// in alive_list) is compared with every variable of the band's target blocks
// [tb0, tb0 + ntb) -- a block form of one step of the paper's workers, each
// comparing itself with its next targets.  A pair is evaluated once: when
// both variables are alive rows of the band (the row's block is a target
// block too) only the lower position evaluates it.  A work-group holds RG
// alive rows (one per wave) against one target block B and one sample chunk;
// the 8 rows of B are staged through LDS and shared by all of its waves.

// Reduce NV per-lane values (NV a power of two, <= 32) to NV totals spread
// over the wave: afterwards lane l holds total number (l >> (6 - log2 NV)) &
// (NV - 1).  Lanes are combined by lane-index bit 5 first and bit 0 last
// whatever NV is, so (addition being commutative) every total is the same
// binary64 value as a full butterfly sum of that value alone.
template <int NV>
__device__ __forceinline__ double reduce_scatter(double (&v)[NV]) {
  const int lane = threadIdx.x & 63;
  int mask = 32;
#pragma unroll
  for (int cnt = NV; cnt > 1; cnt >>= 1) {
    const int half = cnt >> 1;
    const bool hi = lane & mask;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      // select values, not array slots, so that v stays in registers
      const double lo_v = v[i], hi_v = v[half + i];
      const double keep = hi ? hi_v : lo_v;
      const double send = hi ? lo_v : hi_v;
      v[i] = keep + __shfl_xor(send, mask, 64);
    }
    mask >>= 1;
  }
  double x = v[0];
#pragma unroll
  for (; mask >= 1; mask >>= 1) x += __shfl_xor(x, mask, 64);
  return x;
}

template <int NV>
constexpr int log2_of() { return NV <= 1 ? 0 : 1 + log2_of<NV / 2>(); }

// RG alive rows per work-group; each row's 8 targets are split over
// TB / TPW waves of TPW targets each.  The 8 target rows are staged through
// LDS PS samples at a time, double-buffered: the loads of the next stage are
// issued before the current stage is computed, so one barrier per stage
// suffices and the load latency hides behind the arithmetic.
// S is the stored element type: binary64 rows (FP64 and MIXED), or binary32
// rows (FP32 storage, MIXED terms), whose residuals are formed by binary32
// fused multiply-adds with b rounded to binary32.
//
// One item of a band of data set d: row group g of the alive list against
// target block tb0 + tb over sample chunk `chunk` (item = g + nrg (tb + ntb
// chunk)).  The work-group's waves count the pairs they evaluate and
// compute in n_eval / n_comp.
template <bool MIXED, int RG, int TPW, int PS, typename S>
__device__ __forceinline__ void pair_item(const Dev& d, int t, const BandArgs& a, int item, int m, int tb0,
                                          int ntb, unsigned& n_eval, unsigned& n_comp) {
  static_assert(MIXED || sizeof(S) == 8, "binary32 rows take the mixed-precision terms");
  constexpr bool ROW32 = sizeof(S) == 4;
  const int r = rows_left(d, t), p = d.p;
  const int buf = t & 1;
  const S* __restrict__ Z = static_cast<const S*>(d.Z[buf]);
  const int64_t ldz = d.ldz, n = d.n;
  const double* __restrict__ Sig = d.Sig[buf];
  const double* __restrict__ dsc = d.dsc[buf];
  const double* __restrict__ M = d.M;
  const uint8_t* __restrict__ alive = d.alive;
  const int32_t* __restrict__ alive_list = d.alive_list;
  double* __restrict__ P = d.P;
  uint8_t* __restrict__ pend = d.pend;
  const int32_t* __restrict__ idx = d.idx[buf];
  Ctl* ctl = d.ctl;
  const int messaging = d.messaging;
  constexpr int WPR = TB / TPW;     // waves per row
  constexpr int NW = RG * WPR;      // waves per work-group
  constexpr int SPL = PS / 64;      // samples per lane and stage
  constexpr int NT = 64 * NW;       // threads
  constexpr int EV = 16 / (int)sizeof(S);  // elements per 16-byte staging load
  using V = typename std::conditional<ROW32, float4, double2>::type;
  constexpr int NSTG = TB * PS / EV / NT;  // 16-byte loads of the target rows each thread stages
  static_assert(NSTG >= 1 && NSTG * NT == TB * PS / EV, "stage must split evenly over the threads");
  __shared__ S lds[2][TB][PS];  // the 8 rows of target block B, two stages
  __shared__ double s_sc[NW][TPW];   // per-pair scale s = 1/sqrt(1 - b^2)
  __shared__ uint32_t s_mask[NW];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int nrg = (m + RG - 1) / RG;
  const int g = item % nrg;
  const int tb = (item / nrg) % ntb;
  const int chunk = item / (nrg * ntb);
  const int B = tb0 + tb;
  const int q = g * RG + wave / WPR;
  const int j0 = (wave % WPR) * TPW;  // first target of this wave within B
  const int v = q < m ? alive_list[q] : -1;
  // which of the TPW pairs (v, w in B) this wave evaluates (wave-uniform)
  uint32_t mask = 0;
  if (v >= 0) {
    const int bv = v / TB;
    const bool v_in_targets = bv >= tb0 && bv < tb0 + ntb;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int w = B * TB + j0 + j;
      if (w >= r || w == v) continue;
      if (!__builtin_isnan(M[(int64_t)v * p + w])) continue;
      const bool w_row = alive[w] != 0 && v_in_targets;  // w also a row of this band
      // messaging (Sec. 3.1): a pair both of whose variables are rows of the
      // band is evaluated once, by the lower position; without it every row
      // evaluates its own direction
      if (!w_row || v < w || !messaging) mask |= 1u << j;
    }
  }
  mask = __builtin_amdgcn_readfirstlane(mask);
  if (lane == 0) s_mask[wave] = mask;
  __syncthreads();
  int n_act = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) n_act += s_mask[w] ? 1 : 0;
  if (n_act == 0) {  // nothing in this item for any wave (uniform)
    __syncthreads();
    return;
  }

  // per-pair regression coefficient b (correlation of the normalised rows)
  // and scale s = 1/sqrt(1 - b^2) (Eq. var_update); s waits in LDS for the
  // epilogue so it holds no registers during the sample loop
  double bj[TPW];
  float bf[TPW];  // b rounded to binary32 (binary32 rows)
  float ca[TPW], cg[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    bj[j] = 0.0;
    double sj = 1.0;
    if (mask >> j & 1u) {
      const int w = B * TB + j0 + j;
      // symmetric in v and w (Sigma is stored symmetric bit for bit), so a
      // pair gets the same bits whichever of its variables is the row
      const double b = Sig[(int64_t)v * p + w] * (dsc[v] * dsc[w]);
      const double om = 1.0 - b * b;
      if (!(om > DEGEN_EPS)) {
        if (lane == 0) raise_error(ctl, ST_DEGENERATE, idx[v], idx[w]);
      } else {
        bj[j] = b;
        sj = rsqrt(om);
      }
    }
    if (lane == j) s_sc[wave][j] = sj;
    bf[j] = (float)bj[j];
    ca[j] = (float)(-2.0 * 1.4426950408889634074 * sj);
    cg[j] = (float)(-0.5 * 1.4426950408889634074 * sj * sj);
  }

  const int64_t k0 = (int64_t)chunk * a.chunk;
  const int64_t kend = min(n, k0 + (int64_t)a.chunk);
  const int nst = (int)((kend - k0 + PS - 1) / PS);
  const S* zrow = Z + (int64_t)(mask ? v : 0) * ldz;
  // this thread's share of the staged target rows (a target position past
  // the last variable, var >= r, is read from row r - 1, and its pairs are
  // never kept)
  const S* srow[NSTG];
#pragma unroll
  for (int i = 0; i < NSTG; ++i) {
    const int e = i * NT + (int)threadIdx.x;
    const int var = B * TB + e / (PS / EV);
    srow[i] = Z + (int64_t)min(var, r - 1) * ldz + EV * (e % (PS / EV));
  }
  V stg[NSTG];
  S zn[SPL];
  // global loads of one stage into registers.  A stage starts at a multiple
  // of SUB below n, and PS divides SUB, so the whole stage lies inside the
  // row's zero-padded stride ldz = n rounded up to SUB: the loads need no
  // bounds test (samples past n are read as padding and never summed).
  static_assert(SUB % PS == 0, "a stage must end inside the padded row");
  auto load_stage = [&](int64_t ks) {
#pragma unroll
    for (int i = 0; i < NSTG; ++i) stg[i] = *reinterpret_cast<const V*>(srow[i] + ks);
#pragma unroll
    for (int i = 0; i < SPL; ++i) zn[i] = zrow[ks + i * 64 + lane];
  };

  // accumulators: [j][0] lc(r_v), [j][1] g(r_v), [j][2] lc(r_w), [j][3] g(r_w)
  using acc_t = typename std::conditional<MIXED, float, double>::type;
  acc_t acc[TPW][4];
#pragma unroll
  for (int j = 0; j < TPW; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[j][c] = 0;

  load_stage(k0);
  for (int st = 0; st < nst; ++st) {
    const int64_t ks = k0 + (int64_t)st * PS;
    const int cnt = (int)min((int64_t)PS, kend - ks);
    S (*buf)[PS] = lds[st & 1];
#pragma unroll
    for (int i = 0; i < NSTG; ++i) {
      const int e = i * NT + (int)threadIdx.x;
      const int row = e / (PS / EV), c2 = e % (PS / EV);
      // element-wise, so that stg stays in registers
      if constexpr (ROW32)
        *reinterpret_cast<float4*>(&buf[row][EV * c2]) = make_float4(stg[i].x, stg[i].y, stg[i].z, stg[i].w);
      else
        *reinterpret_cast<double2*>(&buf[row][EV * c2]) = make_double2(stg[i].x, stg[i].y);
    }
    S zv[SPL];
#pragma unroll
    for (int i = 0; i < SPL; ++i) zv[i] = zn[i];
    // buf is complete, and every wave has finished the stage that last used
    // the other buffer
    __syncthreads();
    if (st + 1 < nst) load_stage(ks + PS);
    if (mask) {
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        const int k = i * 64 + lane;
        if (k < cnt) {
#pragma unroll
          for (int j = 0; j < TPW; ++j) {
            const S zw = buf[j0 + j][k];
            if constexpr (ROW32) {
              const float rv = __builtin_fmaf(-bf[j], zw, zv[i]);  // r_v^(w) / s
              const float rw = __builtin_fmaf(-bf[j], zv[i], zw);  // r_w^(v) / s
              terms_mixed(rv, ca[j], cg[j], acc[j][0], acc[j][1]);
              terms_mixed(rw, ca[j], cg[j], acc[j][2], acc[j][3]);
            } else {
              const double rv = __builtin_fma(-bj[j], zw, zv[i]);  // r_v^(w) / s
              const double rw = __builtin_fma(-bj[j], zv[i], zw);  // r_w^(v) / s
              if constexpr (MIXED) {
                terms_mixed((float)rv, ca[j], cg[j], acc[j][0], acc[j][1]);
                terms_mixed((float)rw, ca[j], cg[j], acc[j][2], acc[j][3]);
              } else {
                const double sj = s_sc[wave][j];
                double t0 = acc[j][0], t1 = acc[j][1], t2 = acc[j][2], t3 = acc[j][3];
                terms_f64(sj * rv, t0, t1);
                terms_f64(sj * rw, t2, t3);
                acc[j][0] = t0; acc[j][1] = t1; acc[j][2] = t2; acc[j][3] = t3;
              }
            }
          }
        }
      }
    }
  }

  // convert to sum(log cosh u + ln 2) and sum(u exp(-u^2/2)), reduce over the wave
  constexpr int NV = 4 * TPW;
  double vals[NV];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    if constexpr (MIXED) {
      const double sj = s_sc[wave][j];
      vals[4 * j + 0] = (double)acc[j][0] * LN2;
      vals[4 * j + 1] = (double)acc[j][1] * sj;
      vals[4 * j + 2] = (double)acc[j][2] * LN2;
      vals[4 * j + 3] = (double)acc[j][3] * sj;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) vals[4 * j + c] = (double)acc[j][c];
    }
  }
  const double tot = mask ? reduce_scatter<NV>(vals) : 0.0;
  constexpr int SH = 6 - log2_of<NV>();
  if ((lane & ((1 << SH) - 1)) == 0) {
    const int qq = lane >> SH, j = qq >> 2, c = qq & 3;
    if (mask >> j & 1u) {
      const int w = B * TB + j0 + j;
      P[(((int64_t)chunk * p + v) * p + w) * 4 + c] = tot;
      if (messaging) P[(((int64_t)chunk * p + w) * p + v) * 4 + ((c + 2) & 3)] = tot;
    }
  }
  if (chunk == 0 && lane < TPW && (mask >> lane & 1u)) {
    const int w = B * TB + j0 + lane;
    pend[(int64_t)v * p + w] = 1;
    if (messaging) pend[(int64_t)w * p + v] = 1;   // the reverse test is the negation
  }
  if (chunk == 0 && mask) {
    n_eval += (unsigned)__popc(mask);
    n_comp += TPW;
  }
  __syncthreads();  // s_mask, s_sc and lds are reused by the next item
}

// A band of one data set (blockIdx.z of a grid-z launch, or the only one):
// the grid is bounded and each work-group walks its share of the items.
// Work-groups are dealt round-robin over the 8 XCDs, so each XCD takes one
// contiguous eighth of the items (same chunk and target block, different
// row groups) and its work-groups share the XCD's L2.
template <bool MIXED, int RG, int TPW, int PS, typename S>
__device__ __forceinline__ void k_pair_band_body(const Dev& d, int t, BandArgs a) {
  constexpr int NW = RG * (TB / TPW);
  const int r = rows_left(d, t);
  if (r < 2) return;
  Ctl* ctl = d.ctl;
  __shared__ int s_stop, s_m, s_tb0, s_ntb;
  // the stop decision, the alive count and the band are read once and
  // shared, so the whole work-group decides together
  if (threadIdx.x == 0) {
    s_stop = halted(ctl) || ctl->done;
    s_m = ctl->n_alive;
    s_tb0 = ctl->tb_next;
    s_ntb = ctl->ntb_next;
  }
  __syncthreads();
  const int m = s_m;
  if (s_stop) return;
  const int tb0 = s_tb0, ntb = s_ntb;
  const int nrg = (m + RG - 1) / RG;
  const int items = nrg * ntb * d.nchunk;
  const int xcd = blockIdx.x % 8, per_xcd = gridDim.x / 8;
  const int ipx = (items + 7) / 8;
  const int lo = xcd * ipx, hi = min(items, lo + ipx);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  unsigned n_eval = 0, n_comp = 0;  // pairs this wave evaluated / computed
  for (int item = lo + (int)(blockIdx.x / 8); item < hi; item += per_xcd)
    pair_item<MIXED, RG, TPW, PS, S>(d, t, a, item, m, tb0, ntb, n_eval, n_comp);
  // one add per wave, on addresses spread over the slots
  if (lane == 0 && n_comp) {
    const int slot = (int)((blockIdx.x * NW + wave) % PAIR_SLOTS);
    atomicAdd(&d.pair_slots[slot], (unsigned long long)n_eval);
    atomicAdd(&d.pair_slots[PAIR_SLOTS + slot], (unsigned long long)n_comp);
  }
}

// Items of a batch's data set at the current band (0 when it has no band
// running: finished, halted, or its iteration decided).
template <int RG>
__device__ __forceinline__ int band_items(const Dev& d, int t) {
  const Ctl* c = d.ctl;
  if (rows_left(d, t) < 2 || halted(c) || c->done) return 0;
  return (c->n_alive + RG - 1) / RG * c->ntb_next * d.nchunk;
}

// Device work queue over the data sets of a batch.  The grid is persistent
// (about the work-groups the device holds at once) and not tied to any data
// set: a work-group claims QCLAIM items of one data set at a time from that
// set's claim counter (Ctl::q_next), first from the set it worked on last,
// and when that set has no items left it looks, from that set onward, for
// the next set that still has some.  Small or finished data sets therefore
// occupy no work-groups, and the last live sets of an uneven batch get the
// whole device.  The host passes the sets that still have an iteration at
// t (act[0, nact), in order of the iteration they end at, latest first), so
// the search skips the finished ones.  (Counters start at 0 with each band:
// the iteration set-up and every band decision reset them.)
constexpr int QCLAIM = 4;

// The first set, in rotation order from position `start` of act, for which
// has_work(set) holds; -1 if none.  All threads of the group take part.
template <class F>
__device__ int find_set(const int32_t* __restrict__ act, int nact, int start, int* sh_best, F has_work) {
  if (threadIdx.x == 0) *sh_best = 0x7fffffff;
  __syncthreads();
  for (int off = threadIdx.x; off < nact; off += blockDim.x) {
    const int pos = (start + off) % nact;
    if (has_work(act[pos])) {
      atomicMin(sh_best, off);
      break;
    }
  }
  __syncthreads();
  const int best = *sh_best;
  __syncthreads();
  return best == 0x7fffffff ? -1 : (start + best) % nact;
}

template <bool MIXED, int RG, int TPW, int PS, typename S>
__device__ __forceinline__ void k_pair_queue_body(const Dev* __restrict__ devs, const int32_t* __restrict__ act,
                                                  int nact, int t, BandArgs a) {
  constexpr int NW = RG * (TB / TPW);
  __shared__ int s_best, s_i0, s_cnt, s_m, s_tb0, s_ntb;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  if (nact < 1) return;
  int pos = (int)((int64_t)blockIdx.x * nact / gridDim.x);
  int cur_set = -1;
  unsigned n_eval = 0, n_comp = 0;
  auto flush = [&](int k) {
    if (k >= 0 && lane == 0 && n_comp) {
      const int slot = (int)((blockIdx.x * NW + wave) % PAIR_SLOTS);
      atomicAdd(&devs[k].pair_slots[slot], (unsigned long long)n_eval);
      atomicAdd(&devs[k].pair_slots[PAIR_SLOTS + slot], (unsigned long long)n_comp);
    }
    n_eval = n_comp = 0;
  };
  auto has_items = [&](int k) {
    const Dev& d = devs[k];
    const int items = band_items<RG>(d, t);
    return items > 0 && (int)__atomic_load_n(&d.ctl->q_next, __ATOMIC_RELAXED) < items;
  };
  bool fresh = true;   // pos has not been tried since it was chosen
  for (;;) {
    if (!fresh) {
      pos = find_set(act, nact, pos, &s_best, has_items);
      if (pos < 0) break;
    }
    fresh = false;
    const int k = act[pos];
    if (threadIdx.x == 0) {
      const Dev& d = devs[k];
      const int items = band_items<RG>(d, t);
      int i0 = items;
      if (items > 0 && (int)__atomic_load_n(&d.ctl->q_next, __ATOMIC_RELAXED) < items)
        i0 = (int)atomicAdd(&d.ctl->q_next, (uint32_t)QCLAIM);
      s_i0 = i0;
      s_cnt = i0 < items ? min(QCLAIM, items - i0) : 0;
      s_m = d.ctl->n_alive;
      s_tb0 = d.ctl->tb_next;
      s_ntb = d.ctl->ntb_next;
    }
    __syncthreads();
    const int i0 = s_i0, cnt = s_cnt, m = s_m, tb0 = s_tb0, ntb = s_ntb;
    __syncthreads();
    if (cnt == 0) continue;   // this set is exhausted: look for another
    fresh = true;             // try the same set again next
    if (k != cur_set) {
      flush(cur_set);
      cur_set = k;
    }
    for (int item = i0; item < i0 + cnt; ++item)
      pair_item<MIXED, RG, TPW, PS, S>(devs[k], t, a, item, m, tb0, ntb, n_eval, n_comp);
  }
  flush(cur_set);
}

// BATCH selects the descriptor source at compile time, so each instance
// holds one copy of the (register-heavy) body.
template <bool MIXED, int RG, int TPW, int PS, bool BATCH, typename S>
__global__ __launch_bounds__(64 * RG * (TB / TPW)) void k_pair_band(const Dev* __restrict__ devs, const Dev one,
                                                                   int t, BandArgs a) {
  if constexpr (BATCH)
    k_pair_band_body<MIXED, RG, TPW, PS, S>(devs[blockIdx.z], t, a);
  else
    k_pair_band_body<MIXED, RG, TPW, PS, S>(one, t, a);
}

// The batch form: one persistent grid over the device work queue.
template <bool MIXED, int RG, int TPW, int PS, typename S>
__global__ __launch_bounds__(64 * RG * (TB / TPW)) void k_pair_queue(const Dev* __restrict__ devs,
                                                                    const int32_t* __restrict__ act, int nact,
                                                                    int t, BandArgs a) {
  k_pair_queue_body<MIXED, RG, TPW, PS, S>(devs, act, nact, t, a);
}

// Work-group shapes of the pair kernel (results do not depend on them;
// chosen by measurement on MI355X).  Mixed mode: 2 rows per group, each
// row's 8 targets split over 2 waves of 4, 256-sample stages -- small groups
// that the CUs hold several at a time, so the first band of an iteration
// (every row, one target block) and the later bands (few rows, several
// blocks) both spread over the whole device.  The first band's grid may
// take many generations of groups; later bands are bounded to one.  FP64
// mode: one row per group, its 8 targets over 4 waves of 2 (its terms need
// more registers per lane), later bands bounded to two generations.
template <bool MIXED, int RG, int TPW, int PS, typename S>
static int resident_groups() {
  static std::atomic<int> cached{0};
  if (cached.load() == 0) {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pair_band<MIXED, RG, TPW, PS, false, S>,
                                                     64 * RG * (TB / TPW), 0) != hipSuccess ||
        per_cu < 1 || cus < 1) {
      per_cu = 1;
      cus = 256;
    }
    cached.store(per_cu * cus);
  }
  return cached.load();
}

template <bool MIXED, int RG, int TPW, int PS, typename S>
static int groups_per_set(const Batch& b, int max_waves) {
  return std::max(8, max_waves * resident_groups<MIXED, RG, TPW, PS, S>() / b.count);
}

template <bool MIXED, int RG, int TPW, int PS, typename S>
static void launch_pair_shape(const Batch& b, int t, const BandArgs& a, int ntb_hint, hipStream_t s,
                              int max_waves, hipEvent_t ev0, hipEvent_t ev1) {
  const int r = b.p_max - t;
  const int nb = (r + TB - 1) / TB;
  const int ntb = std::max(1, std::min(ntb_hint, nb));  // most target blocks the band can have
  if (r < 2) return;
  const int nrg = (r + RG - 1) / RG;
  // at most max_waves generations of resident work-groups over the batch;
  // sparse bands use one, so no work-group waits for a slot only to find
  // nothing to do
  const int per_set = groups_per_set<MIXED, RG, TPW, PS, S>(b, max_waves);
  const int G = std::min(ntb * b.nchunk_max * nrg, per_set);  // items when every row is alive
  const int grid = (G + 7) / 8 * 8;
  const dim3 g(grid, 1, b.count), blk(64 * RG * (TB / TPW));
  // the events, when given, take the launch's own start and end times, so
  // they add no packets of their own between the kernels
  if (b.count == 1) {
    hipExtLaunchKernelGGL((k_pair_band<MIXED, RG, TPW, PS, false, S>), g, blk, 0, s, ev0, ev1, 0,
                          (const Dev*)nullptr, b.one, t, a);
  } else if (b.queue) {
    // the persistent grid: the work-groups the device holds at once
    const int gq = (resident_groups<MIXED, RG, TPW, PS, S>() + 7) / 8 * 8;
    hipExtLaunchKernelGGL((k_pair_queue<MIXED, RG, TPW, PS, S>), dim3(gq), blk, 0, s, ev0, ev1, 0,
                          (const Dev*)b.dd, b.act, b.active_at(t), t, a);
  } else {
    hipExtLaunchKernelGGL((k_pair_band<MIXED, RG, TPW, PS, true, S>), g, blk, 0, s, ev0, ev1, 0,
                          (const Dev*)b.dd, b.one, t, a);
  }
}

void pair_band_shape(const Batch& b, int& rows_per_group, int& groups) {
  if (b.store32) {
    rows_per_group = 2;
    groups = groups_per_set<true, 2, 4, 256, float>(b, 1);
  } else if (b.mixed) {
    rows_per_group = 2;
    groups = groups_per_set<true, 2, 4, 256, double>(b, 1);
  } else {
    rows_per_group = 1;
    groups = groups_per_set<false, 1, 2, 256, double>(b, 2);
  }
}

hipError_t launch_pair_band(const Batch& b, int t, const BandArgs& a, int dense, int ntb_hint, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
  const int waves = dense ? 1 << 16 : 1;
  if (b.store32)
    launch_pair_shape<true, 2, 4, 256, float>(b, t, a, ntb_hint, s, waves, ev0, ev1);
  else if (b.mixed)
    launch_pair_shape<true, 2, 4, 256, double>(b, t, a, ntb_hint, s, waves, ev0, ev1);
  else
    launch_pair_shape<false, 1, 2, 256, double>(b, t, a, ntb_hint, s, dense ? 1 << 16 : 2, ev0, ev1);
  return hipGetLastError();
}

// ============================================================================
// f3: the paper's baseline mappings of the tests onto the GPU (Sec. 5.3),
// as ablation variants of the pair step (FP64, every ordered pair, no
// threshold and no messaging)
// ============================================================================
// Each computes, for every ordered pair (x, w) of the remaining variables,
// the chunk partial sums that the pair kernel would write with messaging
// off -- sum(log cosh u + ln 2) and sum(u exp(-u^2/2)) of r_x^(w) and of
// r_w^(x), per chunk of `chunk` samples -- and marks the test pending; the
// score kernel then forms the tests exactly as after the pair kernel.  They
// differ only in how the work is mapped:
//   block worker   one work-group per variable x, which takes its tests one
//                  after another, each over all samples with the whole
//                  group (memory O(rn): only the two rows of the test);
//   thread worker  one work-group per variable x, each thread one test,
//                  the thread walking all samples of its pair alone;
//   block compare  one work-group per ordered pair, over all samples.
// The residual and its scale come from the covariance and row scales as in
// the pair kernel (the rows are already centred and scaled), so nothing is
// recomputed per test beyond the sample sums.

// The pair's regression coefficient b and residual scale 1/sqrt(1 - b^2),
// formed as the pair kernel forms them; false for a degenerate pair
// (1 - b^2 <= DEGEN_EPS), which the caller reports.
__device__ __forceinline__ bool baseline_coef(const Dev& d, int t, int x, int w, double& b, double& sc) {
  const int buf = t & 1;
  const int p = d.p;
  const double* dsc = d.dsc[buf];
  b = d.Sig[buf][(int64_t)x * p + w] * (dsc[x] * dsc[w]);
  const double om = 1.0 - b * b;
  if (!(om > DEGEN_EPS)) return false;
  sc = rsqrt(om);
  return true;
}

__device__ __forceinline__ void baseline_degenerate(const Dev& d, int t, int x, int w) {
  raise_error(d.ctl, ST_DEGENERATE, d.idx[t & 1][x], d.idx[t & 1][w]);
}

__device__ __forceinline__ void baseline_store(const Dev& d, int x, int w, int c, double a0, double a1, double a2,
                                               double a3) {
  const int p = d.p;
  double* q = d.P + (((int64_t)c * p + x) * p + w) * 4;
  q[0] = a0;
  q[1] = a1;
  q[2] = a2;
  q[3] = a3;
}

// Test (x, w) by one work-group of 256 threads: per chunk, the threads
// stride over its samples and the four sums are reduced over the group.
__device__ __forceinline__ void baseline_pair_group(const Dev& d, int t, int x, int w, int chunk) {
  __shared__ double sh[4];
  double b = 0.0, sc = 1.0;
  if (!baseline_coef(d, t, x, w, b, sc)) {   // the same for every thread
    if (threadIdx.x == 0) baseline_degenerate(d, t, x, w);
    return;
  }
  const double* Z = static_cast<const double*>(d.Z[t & 1]);
  const double* zx = Z + (int64_t)x * d.ldz;
  const double* zw = Z + (int64_t)w * d.ldz;
  const int64_t n = d.n;
  for (int c = 0; c < d.nchunk; ++c) {
    const int64_t k1 = min(n, (int64_t)(c + 1) * chunk);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int64_t k = (int64_t)c * chunk + threadIdx.x; k < k1; k += 256) {
      const double rv = __builtin_fma(-b, zw[k], zx[k]);   // r_x^(w) / s
      const double rw = __builtin_fma(-b, zx[k], zw[k]);   // r_w^(x) / s
      terms_f64(sc * rv, a0, a1);
      terms_f64(sc * rw, a2, a3);
    }
    a0 = block_sum256(a0, sh);
    a1 = block_sum256(a1, sh);
    a2 = block_sum256(a2, sh);
    a3 = block_sum256(a3, sh);
    if (threadIdx.x == 0) baseline_store(d, x, w, c, a0, a1, a2, a3);
  }
  if (threadIdx.x == 0) d.pend[(int64_t)x * d.p + w] = 1;
}

__device__ __forceinline__ void baseline_count(const Dev& d, unsigned long long pairs, int64_t where) {
  if (pairs == 0) return;
  const int slot = (int)(where % PAIR_SLOTS);
  atomicAdd(&d.pair_slots[slot], pairs);
  atomicAdd(&d.pair_slots[PAIR_SLOTS + slot], pairs);
}

__global__ __launch_bounds__(256) void k_block_worker(const Dev d, int t, int chunk) {
  const int r = rows_left(d, t);
  if (r < 2 || halted(d.ctl) || d.ctl->done) return;
  const int x = blockIdx.x;
  for (int w = 0; w < r; ++w)
    if (w != x) baseline_pair_group(d, t, x, w, chunk);
  if (threadIdx.x == 0) baseline_count(d, (unsigned long long)(r - 1), x);
}

__global__ __launch_bounds__(256) void k_thread_worker(const Dev d, int t, int chunk) {
  const int r = rows_left(d, t);
  if (r < 2 || halted(d.ctl) || d.ctl->done) return;
  const int x = blockIdx.x;
  const double* Z = static_cast<const double*>(d.Z[t & 1]);
  const double* zx = Z + (int64_t)x * d.ldz;
  const int64_t n = d.n;
  unsigned long long pairs = 0;
  for (int w = threadIdx.x; w < r; w += 256) {
    double b = 0.0, sc = 1.0;
    if (w == x) continue;
    if (!baseline_coef(d, t, x, w, b, sc)) {
      baseline_degenerate(d, t, x, w);
      continue;
    }
    const double* zw = Z + (int64_t)w * d.ldz;
    for (int c = 0; c < d.nchunk; ++c) {
      const int64_t k1 = min(n, (int64_t)(c + 1) * chunk);
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (int64_t k = (int64_t)c * chunk; k < k1; ++k) {
        const double rv = __builtin_fma(-b, zw[k], zx[k]);
        const double rw = __builtin_fma(-b, zx[k], zw[k]);
        terms_f64(sc * rv, a0, a1);
        terms_f64(sc * rw, a2, a3);
      }
      baseline_store(d, x, w, c, a0, a1, a2, a3);
    }
    d.pend[(int64_t)x * d.p + w] = 1;
    ++pairs;
  }
  baseline_count(d, pairs, (int64_t)x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_block_compare(const Dev d, int t, int chunk) {
  const int r = rows_left(d, t);
  const int x = blockIdx.y, w = blockIdx.x;
  if (x == w || r < 2 || halted(d.ctl) || d.ctl->done) return;
  baseline_pair_group(d, t, x, w, chunk);
  if (threadIdx.x == 0) baseline_count(d, 1ull, (int64_t)x * r + w);
}

hipError_t launch_pair_baseline(const Batch& b, int t, int strategy, int chunk, hipStream_t s) {
  const int r = b.p_max - t;
  if (r < 2) return hipSuccess;
  if (b.count != 1 || b.store32 || b.mixed) return hipErrorInvalidValue;   // FP64 single searches only
  switch (strategy) {
    case LINGAM_PAIR_BLOCK_WORKER:
      hipLaunchKernelGGL(k_block_worker, dim3(r), dim3(256), 0, s, b.one, t, chunk);
      break;
    case LINGAM_PAIR_THREAD_WORKER:
      hipLaunchKernelGGL(k_thread_worker, dim3(r), dim3(256), 0, s, b.one, t, chunk);
      break;
    case LINGAM_PAIR_BLOCK_COMPARE:
      hipLaunchKernelGGL(k_block_compare, dim3(r, r), dim3(256), 0, s, b.one, t, chunk);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ============================================================================
// a5/a6: tests, scores, threshold state, termination and root
// ============================================================================
// Iteration-level decision after a band, taken by one work-group of 256
// threads: the termination test, the threshold update of a round that ended
// without a root, the root, the next band's threshold state and the
// compacted alive list.  One pass over the scores gives the smallest
// complete score (with its lowest original index) and the smallest incomplete one;
// for a threshold gamma, some complete score is <= gamma iff the first is,
// and some incomplete one iff the second is, so the threshold loop needs no
// further pass.  A band that leaves every score above gamma ends its round
// at once: with no variable below the threshold the round's later bands
// would compare nothing and leave every score as it is, so their decisions
// would see these scores again.  Returns 1 when the round ended.
__device__ int decide_group(const double* __restrict__ S, uint8_t* __restrict__ alive,
                             const uint8_t* __restrict__ complete, int32_t* __restrict__ alive_list, int r,
                             int round_end, int t, double gamma_mult, const int32_t* __restrict__ forced,
                             int forced_len, const int32_t* __restrict__ idx, Ctl* ctl) {
  __shared__ double sh_c[4], sh_i[4];
  __shared__ int sh_ci[4], sh_cix[4], sh_pos[4], sh_cnt[4], sh_has[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int want = t < forced_len ? forced[t] : -1;
  double minc = INFINITY, mini = INFINITY;
  // ci: position of the smallest complete score, cix its original index
  // (ties go to the lowest original index); has: bit 0 some complete row,
  // bit 1 some incomplete row
  int ci = 0x7fffffff, cix = 0x7fffffff, pos = -1, has = 0;
  // the scores and complete flags of the first KC * 256 positions stay in
  // registers for the compaction below
  constexpr int KC = 8;
  double sv[KC];
  bool cv[KC];
  auto visit = [&](int y, double sy, bool cy) {
    if (cy) {
      has |= 1;
      const int iy = idx[y];
      if (sy < minc || (sy == minc && iy < cix)) { minc = sy; ci = y; cix = iy; }
    } else {
      has |= 2;
      mini = fmin(mini, sy);
    }
    if (want >= 0 && idx[y] == want) pos = y;
  };
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int y = tid + 256 * k;
    sv[k] = y < r ? S[y] : INFINITY;
    cv[k] = y < r ? complete[y] != 0 : true;
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int y = tid + 256 * k;
    if (y < r) visit(y, sv[k], cv[k]);
  }
  for (int y = tid + 256 * KC; y < r; y += 256) visit(y, S[y], complete[y] != 0);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double oc = __shfl_xor(minc, off, 64);
    const int oci = __shfl_xor(ci, off, 64), ocix = __shfl_xor(cix, off, 64);
    if (oc < minc || (oc == minc && ocix < cix)) { minc = oc; ci = oci; cix = ocix; }
    mini = fmin(mini, __shfl_xor(mini, off, 64));
    pos = max(pos, __shfl_xor(pos, off, 64));
    has |= __shfl_xor(has, off, 64);
  }
  if (lane == 0) {
    sh_c[wv] = minc; sh_ci[wv] = ci; sh_cix[wv] = cix; sh_i[wv] = mini; sh_pos[wv] = pos; sh_has[wv] = has;
  }
  __syncthreads();
  minc = sh_c[0]; ci = sh_ci[0]; cix = sh_cix[0]; mini = sh_i[0]; pos = sh_pos[0]; has = sh_has[0];
  for (int w = 1; w < 4; ++w) {
    if (sh_c[w] < minc || (sh_c[w] == minc && sh_cix[w] < cix)) { minc = sh_c[w]; ci = sh_ci[w]; cix = sh_cix[w]; }
    mini = fmin(mini, sh_i[w]);
    pos = max(pos, sh_pos[w]);
    has |= sh_has[w];
  }
  // termination: some complete score <= gamma and every incomplete one > gamma;
  // a round that ends with every score above gamma raises gamma by c
  double gamma = ctl->gamma;
  int done = 0;
  for (int guard = 0; guard < 4096; ++guard) {
    const bool cand = (has & 1) && minc <= gamma;
    const bool blocked = (has & 2) && mini <= gamma;
    if (cand && !blocked) { done = 1; break; }
    if (!cand && !blocked) {
      round_end = 1;
      gamma = gamma > 0.0 ? gamma * gamma_mult : 1e-300;
      continue;
    }
    break;
  }
  const int root = !done ? -1 : (want >= 0 ? pos : (ci == 0x7fffffff ? -1 : ci));
  // threshold state for the next band and the compacted alive list, in
  // ascending position.  The list holds the variables below the threshold
  // that still have a test to evaluate: a complete variable has none, so it
  // would bring only items that leave at their mask test, and its score no
  // longer changes (it still counts for the termination test above, which
  // reads every score).
  int base = 0;
  auto compact = [&](int y, double sy, bool cy) {
    const int a = y < r && sy <= gamma && !cy ? 1 : 0;
    if (y < r) alive[y] = (uint8_t)a;
    const unsigned long long bal = __ballot(a);
    if (lane == 0) sh_cnt[wv] = __popcll(bal);
    __syncthreads();
    int before = base;
    for (int w = 0; w < wv; ++w) before += sh_cnt[w];
    before += __popcll(bal & ((1ull << lane) - 1ull));
    if (a) alive_list[before] = y;
    base += (sh_cnt[0] + sh_cnt[1]) + (sh_cnt[2] + sh_cnt[3]);
    __syncthreads();
  };
#pragma unroll
  for (int k = 0; k < KC; ++k)
    if (256 * k < r) compact(tid + 256 * k, sv[k], cv[k]);
  for (int y0 = 256 * KC; y0 < r; y0 += 256) {
    const int y = y0 + tid;
    compact(y, y < r ? S[y] : INFINITY, y < r ? complete[y] != 0 : true);
  }
  if (tid == 0) {
    ctl->gamma = gamma;
    ctl->n_alive = base;
    if (done) {
      if (root < 0) {
        raise_error(ctl, ST_INVALID, -1, -1);
      } else {
        ctl->root = root;
        ctl->last_root_S = S[root];
        ctl->done = 1;
      }
    } else if (round_end) {
      ctl->round += 1;
    }
    ctl->bands_total += 1;
    ctl->iter_bands += 1;
  }
  return round_end;
}

// The rows whose tests can have changed in the current band: the variables
// of the band's target blocks, then the alive variables outside them.  Row
// index qrow of [0, band_rows) maps to a position, or to -1 (an alive
// variable that is also a target).
struct BandRows {
  int t_lo, t_hi, m, rows;
};

__device__ __forceinline__ BandRows band_rows(const Dev& d, int t) {
  const int r = rows_left(d, t);
  const Ctl* c = d.ctl;
  BandRows b;
  b.t_lo = c->tb_next * TB;
  b.t_hi = min(r, (c->tb_next + c->ntb_next) * TB);
  b.m = c->n_alive;
  b.rows = (b.t_hi - b.t_lo) + b.m;
  return b;
}

__device__ __forceinline__ int band_row(const Dev& d, const BandRows& br, int qrow) {
  if (qrow < br.t_hi - br.t_lo) return br.t_lo + qrow;
  const int y = d.alive_list[qrow - (br.t_hi - br.t_lo)];
  return (y < br.t_lo || y >= br.t_hi) ? y : -1;
}

// Row x of the band: the pending tests from the chunk partial sums, then
// the row's score S_x recomputed over all its tests in ascending original
// index of the other variable (so its bits do not depend on positions), its
// rounding bound and its complete flag.
// In the mixed modes it also forms the rounding bound eps of every new test
// (the sum of the bounds of its four entropies) and the bound of the row's
// score: a test moved by at most eps changes min(0, M)^2 by at most
// 2 |min(0, M)| eps + 3 eps^2, and not at all when M >= eps.
//
// W = 256: the whole work-group scores the row; thread v takes the tests at
// v, v + 256, ... and the four wave sums are added pairwise.  W = 64: one
// wave scores the row and each lane keeps the four partial sums that
// threads lane, lane + 64, lane + 128 and lane + 192 of the work-group form,
// reduced in the same order, so both forms give the same bits.  The wave
// form scores four rows of a work-group at once with no barrier; short rows
// use it.
struct RowAcc {
  double s = 0.0, es = 0.0, esp = 0.0;
};

template <int W>
__device__ __forceinline__ void score_row(const Dev& d, int t, int x) {
  static_assert(W == 64 || W == 256, "a row is scored by one wave or by the work-group");
  constexpr int K = 256 / W;  // partial sums per thread
  const int r = rows_left(d, t), p = d.p;
  const int buf = t & 1;
  double* __restrict__ M = d.M;
  uint8_t* __restrict__ pend = d.pend;
  const double* __restrict__ P = d.P;
  const double* __restrict__ H = d.H;
  const int32_t* __restrict__ ord = d.ord[buf];
  const int nchunk = d.nchunk;
  const double n = (double)d.n;
  const int mixed = d.mixed, store32 = d.store32;
  const double* __restrict__ dsc = d.dsc[buf];
  double* __restrict__ Meps = d.Meps;
  double* __restrict__ Mepsp = d.Mepsp;
  const double* __restrict__ eH = d.eH;
  const double* __restrict__ eHp = d.eHp;
  const double hx = H[x];
  const double* sig = d.Sig[buf] + (int64_t)x * p;
  const double dx = dsc[x];
  int incomplete = 0;
  // test (x, w): a pending one is formed from its chunk partials (a second,
  // dependent fetch after the flag, the stored test and its bound), then it
  // is added to the row's score and bounds
  auto score_test = [&](int w, RowAcc& acc) {
    const int64_t o = (int64_t)x * p + w;
    const uint8_t pd = pend[o];
    double mv = M[o], ev = mixed ? Meps[o] : 0.0, evp = mixed ? Mepsp[o] : 0.0;
    if (pd) {
      // the chunk partials in chunk order; eight chunks' loads are issued
      // before their sums, so a test waits for one memory round trip per
      // eight chunks (a chunk past the last re-reads the last and is not
      // added)
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      const double* q0 = P + ((int64_t)x * p + w) * 4;
      const int64_t cstride = (int64_t)p * p * 4;
      for (int c0 = 0; c0 < nchunk; c0 += 8) {
        double4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          v[k] = *reinterpret_cast<const double4*>(q0 + (int64_t)min(c0 + k, nchunk - 1) * cstride);
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (c0 + k < nchunk) {
            a0 += v[k].x; a1 += v[k].y; a2 += v[k].z; a3 += v[k].w;
          }
      }
      const double h_rx = happ_from_sums(a0, a1, n);  // H(r_x^(w))
      const double h_rw = happ_from_sums(a2, a3, n);  // H(r_w^(x))
      mv = (H[w] + h_rx) - (hx + h_rw);               // Eq. (Itest)
      M[o] = mv;
      pend[o] = 0;
      if (mixed) {
        double sin = 0.0;
        if (store32) {
          const double b = sig[w] * (dx * dsc[w]);   // as the pair kernel forms it
          sin = 1.0 / sqrt(1.0 - b * b);
        }
        ev = (eH[x] + eH[w]) + (happ_err_mixed(a0, a1, n, sin) + happ_err_mixed(a2, a3, n, sin));
        evp = (eHp[x] + eHp[w]) + (happ_err_prob(a0, a1, n, sin) + happ_err_prob(a2, a3, n, sin));
        Meps[o] = ev;
        Mepsp[o] = evp;
      }
    } else if (__builtin_isnan(mv)) {
      ev = evp = 0.0;   // not evaluated (its bound slots hold an earlier iteration's values)
    }
    if (__builtin_isnan(mv)) {
      incomplete = 1;
    } else {
      const double neg = mv < 0.0 ? mv : 0.0;
      acc.s += neg * neg;
      if (mv < ev) acc.es += 2.0 * (-neg) * ev + 3.0 * ev * ev;
      if (mv < evp) acc.esp += 2.0 * (-neg) * evp + 3.0 * evp * evp;
    }
  };
  const int v0 = W == 256 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  RowAcc acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    for (int q = v0 + 64 * k; q < r; q += 256) {
      const int w = ord[q];
      if (w != x) score_test(w, acc[k]);
    }
  double s, es = 0.0, esp = 0.0;
  if constexpr (W == 256) {
    __shared__ double sh[4];
    __shared__ int shi[4];
    s = block_sum256(acc[0].s, sh);
    if (mixed) {
      es = block_sum256(acc[0].es, sh);
      esp = block_sum256(acc[0].esp, sh);
    }
    incomplete = block_or256(incomplete, shi);
  } else {
    s = (wave_sum(acc[0].s) + wave_sum(acc[1].s)) + (wave_sum(acc[2].s) + wave_sum(acc[3].s));
    if (mixed) {
      es = (wave_sum(acc[0].es) + wave_sum(acc[1].es)) + (wave_sum(acc[2].es) + wave_sum(acc[3].es));
      esp = (wave_sum(acc[0].esp) + wave_sum(acc[1].esp)) + (wave_sum(acc[2].esp) + wave_sum(acc[3].esp));
    }
    incomplete = __any(incomplete) ? 1 : 0;
  }
  if (v0 == 0) {
    d.S[x] = s;
    d.eT[x] = es;
    d.eTp[x] = esp;
    d.complete[x] = incomplete ? 0 : 1;
  }
}

// The iteration-level decision after a band of data set d (one work-group
// of 256 threads, once every row of the band is scored): termination,
// threshold update, root, threshold state and the next band's target
// blocks; then the band counters are cleared for the next launch.
__device__ __forceinline__ void band_decision(const Dev& d, int t, const BandArgs& a, double gamma_mult) {
  const int r = rows_left(d, t);
  const int nb = (r + TB - 1) / TB;
  const int buf = t & 1;
  Ctl* ctl = d.ctl;
  __shared__ int s_tb0, s_ntb;
  if (threadIdx.x == 0) {
    s_tb0 = ctl->tb_next;
    s_ntb = ctl->ntb_next;
  }
  __syncthreads();
  const int tb0 = s_tb0, ntb = s_ntb;
  // the last band of the round, or a band after which no variable is left
  // below the threshold
  const int round_end = decide_group(d.S, d.alive, d.complete, d.alive_list, r, tb0 + ntb >= nb ? 1 : 0, t,
                                     gamma_mult, d.forced, d.forced_len, d.idx[buf], ctl);
  if (threadIdx.x == 0 && !ctl->done && ctl->status == ST_OK) {
    // the next band: after the end of a round every block at once; within
    // round 0 the following blocks, as many as bring the band near the
    // target work for the rows still below the threshold
    if (round_end) {
      ctl->tb_next = 0;
      ctl->ntb_next = nb;
    } else {
      const int left = nb - (tb0 + ntb);
      int k = d.band_k0;
      if (d.band_adapt) {
        const int m_next = max(ctl->n_alive, 1);
        const double want = a.band_target / ((double)TB * (double)m_next * (double)d.n);
        // whole rounds of the work-groups: a target block brings one item
        // per row group and chunk, and a band whose items overrun a round
        // by a few leaves most groups idle for a second one
        const int per_block = (m_next + a.rows_per_group - 1) / a.rows_per_group * d.nchunk;
        const int fill = a.groups / per_block;  // blocks that fill one round
        if (fill >= 1)
          k = fill * max(1, (int)ceil(want / (double)fill));
        else
          k = max(k, (int)ceil(want));
        if (want >= (double)left) k = left;
      }
      ctl->tb_next = tb0 + ntb;
      ctl->ntb_next = min(k, left);
    }
  }
  if (threadIdx.x == 0) {
    // ready for the next band: its pair launch starts claiming items at 0
    // (no pair launch is running now)
    ctl->arrivals = 0;
    ctl->q_next = 0;
  }
}

// One data set (grid z, or alone): the work-groups walk the band's rows;
// the last work-group to finish takes the decision.  Each group publishes
// its scores (release) before it counts itself in; the last one acquires
// them.  Nothing waits, so no group can be held up.
__device__ __forceinline__ void k_score_body(const Dev& d, int t, BandArgs a, double gamma_mult) {
  const int r = rows_left(d, t);
  if (r < 2) return;
  Ctl* ctl = d.ctl;
  __shared__ int s_stop, s_last, s_wrote;
  __shared__ BandRows s_br;
  if (threadIdx.x == 0) {
    s_stop = halted(ctl) || ctl->done;
    s_wrote = 0;
    s_br = band_rows(d, t);
  }
  __syncthreads();
  if (s_stop) return;
  const BandRows br = s_br;
  if (r <= a.score_wave_rows) {
    // one row per wave, four per work-group
    const int wv = threadIdx.x >> 6;
    for (int qrow = blockIdx.x * 4 + wv; qrow < br.rows; qrow += gridDim.x * 4) {
      const int x = band_row(d, br, qrow);
      if (x < 0) continue;  // uniform over the wave
      score_row<64>(d, t, x);
      if ((threadIdx.x & 63) == 0) s_wrote = 1;
    }
  } else {
    for (int qrow = blockIdx.x; qrow < br.rows; qrow += gridDim.x) {
      const int x = band_row(d, br, qrow);
      if (x < 0) continue;  // uniform over the work-group
      score_row<256>(d, t, x);
      if (threadIdx.x == 0) s_wrote = 1;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_wrote) __threadfence();
    const unsigned prev = atomicAdd(&ctl->arrivals, 1u);
    s_last = prev == gridDim.x - 1 ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  band_decision(d, t, a, gamma_mult);
}

__global__ __launch_bounds__(256) void k_score(const Dev* __restrict__ devs, const Dev one, int t, BandArgs a,
                                               double gamma_mult) {
  if (devs)
    k_score_body(devs[blockIdx.z], t, a, gamma_mult);
  else
    k_score_body(one, t, a, gamma_mult);
}

hipError_t launch_score(const Batch& b, int t, const BandArgs& band, double gamma_mult, int dense, int ntb_hint,
                        hipStream_t s) {
  const int r = b.p_max - t;
  if (r < 2) return hipSuccess;
  // A batch has many more rows than a launch has work-groups, so one wave
  // per row (four rows per group at once) keeps more rows in flight; one
  // search has few rows per group and scores each with the whole group,
  // which halves a row's latency.  Both forms give the same bits.
  BandArgs a = band;
  a.score_wave_rows = b.count > 1 ? 1 << 30 : 0;
  const int nb = (r + TB - 1) / TB;
  // rows when every variable is alive; after the first band of an iteration
  // few are, and a smaller grid keeps idle groups from filling the launch.
  // A batch scores in grid slices also when its pair items run on the work
  // queue: a slice needs no claims, and a finished set's groups return at
  // once (measured faster than claiming rows from a queue).
  // rows scored one per wave go four to a work-group
  const int rows = std::min(r, std::max(1, std::min(ntb_hint, nb)) * TB) + r;
  const int groups = r <= a.score_wave_rows ? (rows + 3) / 4 : rows;
  // every group of a set publishes its scores to the set's decision with a
  // device-wide fence, whose cost grows with the number of groups: a large
  // batch keeps about 1024 groups in all
  const int cap = b.count == 1 ? (dense ? 512 : 256)
                               : std::max(4, std::min((dense ? 512 : 256) / std::min(b.count, 16), 1024 / b.count));
  hipLaunchKernelGGL(k_score, dim3(std::min(groups, cap), 1, b.count), dim3(256), 0, s, DEVS(b), t, a, gamma_mult);
  return hipGetLastError();
}

// ============================================================================
// initial contents of a search's buffers (one launch for every data set)
// ============================================================================
// Tests, records and results "not evaluated" (NaN) or empty, the positions
// and original-index ranks the identity, the pair counters zero, the zero
// padding past n of the second row buffer (the Gram sums over whole
// 64-sample stages), and the control block.
template <typename S>
__device__ __forceinline__ void init_set_body(const Dev& d) {
  const int64_t P = d.p, pp = P * P;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  const double nan = __builtin_nan("");
  for (int64_t e = g; e < pp; e += step) {
    d.M[e] = nan;
    d.Tall[e] = nan;
    d.Hall[e] = nan;
    d.Terr[e] = nan;
    d.Terrp[e] = nan;
    d.Tstate[e] = 0;
    d.pend[e] = 0;
  }
  if (d.Mrec)
    for (int64_t e = g; e < (int64_t)d.rec * pp; e += step) d.Mrec[e] = nan;
  for (int64_t i = g; i < P; i += step) {
    d.idx[0][i] = (int32_t)i;
    d.ord[0][i] = (int32_t)i;
    d.order[i] = -1;
  }
  for (int64_t e = g; e < 2 * PAIR_SLOTS; e += step) d.pair_slots[e] = 0ull;
  const int64_t pad = d.ldz - d.n;
  S* z1 = static_cast<S*>(d.Z[1]);
  for (int64_t e = g; e < P * pad; e += step) z1[(e / pad) * d.ldz + d.n + e % pad] = (S)0;
  if (g == 0) {
    Ctl c{};
    c.halt_iter = -1;
    c.root = -1;
    c.bad_i = c.bad_j = -1;
    *d.ctl = c;
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_init_set(const Dev* __restrict__ devs, const Dev one) {
  if (devs)
    init_set_body<S>(devs[blockIdx.z]);
  else
    init_set_body<S>(one);
}

hipError_t launch_init_sets(const Batch& b, hipStream_t s) {
  const int64_t P = b.p_max;
  const int64_t work = std::max<int64_t>(P * P, P * 256);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024 / std::min(b.count, 16), (work + 255) / 256));
  if (b.store32)
    hipLaunchKernelGGL(k_init_set<float>, dim3(blocks, 1, b.count), dim3(256), 0, s, DEVS(b));
  else
    hipLaunchKernelGGL(k_init_set<double>, dim3(blocks, 1, b.count), dim3(256), 0, s, DEVS(b));
  return hipGetLastError();
}

// Sum the spread pair counters of every data set into slots 0 (evaluated)
// and 1 (computed), for the host to read with its results.
__device__ __forceinline__ void sum_slots_body(const Dev& d) {
  __shared__ unsigned long long sh[2][4];
  unsigned long long ev = 0ull, comp = 0ull;
  for (int k = threadIdx.x; k < PAIR_SLOTS; k += 256) {
    ev += d.pair_slots[k];
    comp += d.pair_slots[PAIR_SLOTS + k];
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    ev += __shfl_xor(ev, m, 64);
    comp += __shfl_xor(comp, m, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = ev;
    sh[1][threadIdx.x >> 6] = comp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d.pair_slots[0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    d.pair_slots[1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
  }
}

__global__ __launch_bounds__(256) void k_sum_slots(const Dev* __restrict__ devs, const Dev one) {
  if (devs)
    sum_slots_body(devs[blockIdx.z]);
  else
    sum_slots_body(one);
}

hipError_t launch_sum_slots(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_slots, dim3(1, 1, b.count), dim3(256), 0, s, DEVS(b));
  return hipGetLastError();
}

__global__ void k_window_reset(const Dev* __restrict__ devs, const Dev one) {
  Ctl* ctl = devs ? devs[blockIdx.z].ctl : one.ctl;
  ctl->win_bands = 0;
}

// Clear the per-window band maximum of every data set (read by the host).
hipError_t launch_window_reset(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_window_reset, dim3(1, 1, b.count), dim3(1), 0, s, DEVS(b));
  return hipGetLastError();
}

__device__ __forceinline__ void k_record_M_body(const Dev& d, int t) {
  const int r = rows_left(d, t), p = d.p;
  if (r < 2 || t >= d.rec || halted(d.ctl)) return;
  const double* __restrict__ M = d.M;
  const int32_t* __restrict__ idx = d.idx[t & 1];
  double* __restrict__ Mrec = d.Mrec + (int64_t)t * p * p;
  const int64_t total = (int64_t)r * r;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e / r), w = (int)(e % r);
    Mrec[(int64_t)idx[x] * p + idx[w]] = M[(int64_t)x * p + w];
  }
}

__global__ void k_record_M(const Dev* __restrict__ devs, const Dev one, int t) {
  if (devs)
    k_record_M_body(devs[blockIdx.z], t);
  else
    k_record_M_body(one, t);
}

hipError_t launch_record_M(const Batch& b, int t, hipStream_t s) {
  const int r = b.p_max - t;
  if (r < 2) return hipSuccess;
  const int64_t total = (int64_t)r * r;
  int blocks = (int)std::min<int64_t>(1024, (total + 255) / 256);
  hipLaunchKernelGGL(k_record_M, dim3(std::max(blocks, 1), 1, b.count), dim3(256), 0, s, DEVS(b), t);
  return hipGetLastError();
}

// ============================================================================
// end of an iteration: record K, T, H; flag an iteration that is not finished
// ============================================================================
__device__ __forceinline__ void k_finish_iter_body(const Dev& d, int t) {
  const int r = rows_left(d, t), p = d.p;
  Ctl* ctl = d.ctl;
  if (r < 2 || halted(ctl)) return;
  const int32_t* __restrict__ idx = d.idx[t & 1];
  const double* __restrict__ S = d.S;
  const uint8_t* __restrict__ complete = d.complete;
  const double* __restrict__ H = d.H;
  const double* __restrict__ eT = d.eT;
  int32_t* order = d.order;
  double* Tall = d.Tall;
  uint8_t* Tstate = d.Tstate;
  double* Hall = d.Hall;
  double* Terr = d.Terr;
  if (!ctl->done) {
    __syncthreads();
    if (threadIdx.x == 0) {
      ctl->halt_iter = t;
      atomicExch(&ctl->halt, 1);
    }
    return;
  }
  for (int y = threadIdx.x; y < r; y += 256) {
    const int64_t o = (int64_t)t * p + idx[y];
    Tall[o] = -S[y];
    Tstate[o] = complete[y] ? 1 : 2;
    Hall[o] = H[y];
    Terr[o] = eT[y];
    d.Terrp[o] = d.eTp[y];
  }
  if (threadIdx.x == 0) {
    order[t] = idx[ctl->root];
    ctl->rounds_total += (unsigned long long)(ctl->round + 1);
    ctl->win_bands = max(ctl->win_bands, ctl->iter_bands);
  }
}

// ============================================================================
// a7: UpdateData and UpdateCovMat (Sec. 3.4), compacting out the root
// ============================================================================
// Positions of the survivors for the next iteration, once the root is
// known: the new position of a variable is the rank of (S, original index)
// among the remaining variables other than the root, so the next iteration
// starts its threshold rounds with the variables that scored best in this
// one.  Their rank by original index alone gives the next iteration's
// canonical order (ord).  With more than RANK_MAX rows the positions keep
// the original order (every earlier iteration had more rows, so they are
// still in it).
constexpr int RANK_MAX = 16384;
constexpr int RANK_TILE = 1024;
constexpr int RANK_SPLIT = 8;                 // threads per row, each counting a share of the others
constexpr int RANK_ROWS = 256 / RANK_SPLIT;   // rows per work-group

__device__ __forceinline__ void k_rank_body(const Dev& d, int t) {
  const int r = rows_left(d, t);
  const Ctl* ctl = d.ctl;
  if (r < 2 || halted(ctl) || !ctl->done) return;
  const int buf = t & 1;
  const double* __restrict__ S = d.S;
  const int32_t* __restrict__ idx = d.idx[buf];
  int32_t* __restrict__ perm = d.perm;
  int32_t* __restrict__ ordn = d.ord[buf ^ 1];
  const int root = ctl->root;
  const int sub = threadIdx.x % RANK_SPLIT;
  const int w = blockIdx.x * RANK_ROWS + threadIdx.x / RANK_SPLIT;  // old position
  const bool mine = w < r && w != root;
  if (r > RANK_MAX) {
    if (mine && sub == 0) {
      const int wn = w - (w > root ? 1 : 0);
      perm[wn] = w;
      ordn[wn] = wn;
    }
    return;
  }
  __shared__ double sh_s[RANK_TILE];
  __shared__ int sh_i[RANK_TILE];
  const double sw = mine ? S[w] : 0.0;
  const int iw = mine ? idx[w] : 0;
  int rs = 0, ri = 0;
  for (int u0 = 0; u0 < r; u0 += RANK_TILE) {
    const int cnt = min(RANK_TILE, r - u0);
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      sh_s[k] = S[u0 + k];
      sh_i[k] = idx[u0 + k];
    }
    __syncthreads();
    if (mine) {
      for (int k = sub; k < cnt; k += RANK_SPLIT) {
        const int u = u0 + k;
        if (u == root || u == w) continue;
        const double su = sh_s[k];
        const int iu = sh_i[k];
        rs += (su < sw || (su == sw && iu < iw)) ? 1 : 0;
        ri += iu < iw ? 1 : 0;
      }
    }
  }
  // the RANK_SPLIT threads of a row are consecutive lanes of one wave
#pragma unroll
  for (int m = 1; m < RANK_SPLIT; m <<= 1) {
    rs += __shfl_xor(rs, m, 64);
    ri += __shfl_xor(ri, m, 64);
  }
  if (mine && sub == 0) {
    perm[rs] = w;
    ordn[ri] = rs;
  }
}

__global__ __launch_bounds__(256) void k_rank(const Dev* __restrict__ devs, const Dev one, int t) {
  if (devs)
    k_rank_body(devs[blockIdx.z], t);
  else
    k_rank_body(one, t);
}

// UpdateData for one segment of one new row (blockIdx.y = new position,
// blockIdx.x = segment).  With want_h (no Gram refresh before the next
// iteration) it also sums the new row's entropy terms over its samples, in
// the mode's precision (binary32 lane sums of at most 32 terms in the mixed
// mode), for the next iteration's entropy.
template <bool MIXED, typename S>
__device__ __forceinline__ void k_update_rows_body(const Dev& d, int t, int want_h) {
  const int r = rows_left(d, t), p = d.p;
  const Ctl* ctl = d.ctl;
  const int64_t ldz = d.ldz, n = d.n;
  const int segs = entropy_segments_of(n);
  if (r < 2 || (int)blockIdx.y >= r - 1 || (int)blockIdx.x >= segs || halted(ctl) || !ctl->done) return;
  const int buf = t & 1;
  const S* __restrict__ Z = static_cast<const S*>(d.Z[buf]);
  S* __restrict__ Zn = static_cast<S*>(d.Z[buf ^ 1]);
  const double* __restrict__ Sig = d.Sig[buf];
  const double* __restrict__ dsc = d.dsc[buf];
  const int root = ctl->root;
  const int wn = blockIdx.y;                  // new position
  const int w = d.perm[wn];                   // old position
  const double dw = dsc[w], dr = dsc[root];
  const double b = Sig[(int64_t)w * p + root] * dw * dr;   // correlation of the normalised rows
  const double om = 1.0 - b * b;
  // every pair passed 1 - b^2 > 1e-12 at the iteration's start; this guard
  // only keeps a rounding difference from dividing by zero
  if (!(om > 0.0)) {
    if (threadIdx.x == 0) raise_error(const_cast<Ctl*>(ctl), ST_DEGENERATE, d.idx[buf][w], d.idx[buf][root]);
    return;
  }
  const double sc = 1.0 / sqrt(om);
  const S* zr = Z + (int64_t)root * ldz;
  const S* zw = Z + (int64_t)w * ldz;
  S* zo = Zn + (int64_t)wn * ldz;
  // two adjacent samples per thread and step, moved with one vector load
  // per row and one vector store (rows start 16-byte aligned, and a sample
  // at n, read as the second of a pair, lies in the row's padding and is
  // neither stored nor summed)
  using V2 = typename std::conditional<sizeof(S) == 8, double2, float2>::type;
  const int64_t step2 = (int64_t)segs * 512;
  const int64_t k0 = 2 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  // binary64 arithmetic in every mode; binary32 rows are rounded once, on the store
  auto update2 = [&](int64_t k, double& z0, double& z1) {
    const V2 vw = *reinterpret_cast<const V2*>(zw + k), vr = *reinterpret_cast<const V2*>(zr + k);
    z0 = ((double)vw.x - b * (double)vr.x) * sc;   // the rows are stored normalised
    z1 = ((double)vw.y - b * (double)vr.y) * sc;
    if (k + 1 < n) {
      V2 o;
      o.x = (S)z0;
      o.y = (S)z1;
      *reinterpret_cast<V2*>(zo + k) = o;
    } else {
      zo[k] = (S)z0;
    }
  };
  if (!want_h) {
    for (int64_t k = k0; k < n; k += step2) {
      double z0, z1;
      update2(k, z0, z1);
    }
    return;
  }
  // The even and the odd sample of each pair have sums of their own: a lane
  // then accumulates the samples it did when it took one at a time, in the
  // same order (terms that cancel exactly in exact arithmetic, +-c, still
  // cancel exactly; a fused multiply-add adding -c to a rounded +c would
  // leave the product's rounding error)
  double lc = 0.0, g = 0.0, lc1 = 0.0, g1 = 0.0;
  int64_t k = k0;
  if constexpr (MIXED) {
    const float ca = -2.0f * LOG2E_F, cg = -0.5f * LOG2E_F;
    while (k < n) {
      // binary32 lane sums of at most 32 terms
      float flc = 0.f, fg = 0.f, flc1 = 0.f, fg1 = 0.f;
      for (int c = 0; c < 32 && k < n; ++c, k += step2) {
        double z0, z1;
        update2(k, z0, z1);
        terms_mixed((float)z0, ca, cg, flc, fg);   // the value the row holds
        if (k + 1 < n) terms_mixed((float)z1, ca, cg, flc1, fg1);
      }
      lc += (double)flc * LN2;
      g += (double)fg;
      lc1 += (double)flc1 * LN2;
      g1 += (double)fg1;
    }
  } else {
    for (; k < n; k += step2) {
      double z0, z1;
      update2(k, z0, z1);
      terms_f64(z0, lc, g);
      if (k + 1 < n) terms_f64(z1, lc1, g1);
    }
  }
  lc += lc1;
  g += g1;
  __shared__ double sh[4];
  lc = block_sum256(lc, sh);
  g = block_sum256(g, sh);
  if (threadIdx.x == 0) {
    double* hp = d.Hp + ((int64_t)wn * ENT_SEGS + blockIdx.x) * 2;
    hp[0] = lc;
    hp[1] = g;
  }
}

template <bool MIXED, typename S>
__global__ __launch_bounds__(256) void k_update_rows(const Dev* __restrict__ devs, const Dev one, int t,
                                                     int want_h) {
  if (devs)
    k_update_rows_body<MIXED, S>(devs[blockIdx.z], t, want_h);
  else
    k_update_rows_body<MIXED, S>(one, t, want_h);
}

// Work-group 0 first records the iteration's results (or halts an iteration
// the queued bands did not finish); then every group takes its share of
// UpdateCovMat.
__device__ __forceinline__ void k_update_sigma_body(const Dev& d, int t, int recursion) {
  const int r = rows_left(d, t), p = d.p;
  if (blockIdx.x == 0) k_finish_iter_body(d, t);
  const Ctl* ctl = d.ctl;
  if (r < 2 || halted(ctl) || !ctl->done) return;
  const int buf = t & 1;
  const double* __restrict__ Sig = d.Sig[buf];
  double* __restrict__ Sn = d.Sig[buf ^ 1];
  const double* __restrict__ dsc = d.dsc[buf];
  double* __restrict__ dscn = d.dsc[buf ^ 1];
  const int32_t* __restrict__ idx = d.idx[buf];
  int32_t* __restrict__ idxn = d.idx[buf ^ 1];
  const int root = ctl->root;
  const int rn = r - 1;
  const int64_t total = (int64_t)rn * rn;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int32_t* __restrict__ perm = d.perm;
  if (gid < rn) {
    const int w = perm[gid];
    idxn[gid] = idx[w];
    if (recursion) dscn[gid] = 1.0;  // the recursion's rows are unit-variance by construction
  }
  if (!recursion) return;
  for (int64_t e = gid; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int an = (int)(e / rn), bn = (int)(e % rn);
    const int a = perm[an], b = perm[bn];
    double val;
    if (an == bn) {
      val = 1.0;
    } else {
      const double da = dsc[a], db = dsc[b], dr = dsc[root];
      const double ba = Sig[(int64_t)a * p + root] * da * dr, bb = Sig[(int64_t)b * p + root] * db * dr;
      const double bab = Sig[(int64_t)a * p + b] * (da * db);   // symmetric in a and b
      // both factors are positive: every pair passed 1 - b^2 > 1e-12 at the
      // iteration's start (the row update guards the root's pairs)
      val = (bab - ba * bb) / (sqrt(fmax(1.0 - ba * ba, DEGEN_EPS)) * sqrt(fmax(1.0 - bb * bb, DEGEN_EPS)));
    }
    Sn[(int64_t)an * p + bn] = val;
  }
}

__global__ __launch_bounds__(256) void k_update_sigma(const Dev* __restrict__ devs, const Dev one, int t, int recursion) {
  if (devs)
    k_update_sigma_body(devs[blockIdx.z], t, recursion);
  else
    k_update_sigma_body(one, t, recursion);
}

hipError_t launch_iter_end(const Batch& b, int t, int refresh, hipStream_t s) {
  const int rn = b.p_max - t - 1;
  if (rn <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rank, dim3((rn + 1 + RANK_ROWS - 1) / RANK_ROWS, 1, b.count), dim3(256), 0, s, DEVS(b), t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int xblocks = entropy_segments_of(b.n_max);
  const int want_h = refresh ? 0 : 1;
  const dim3 ug(xblocks, rn, b.count);
  if (b.store32)
    hipLaunchKernelGGL((k_update_rows<true, float>), ug, dim3(256), 0, s, DEVS(b), t, want_h);
  else if (b.mixed)
    hipLaunchKernelGGL((k_update_rows<true, double>), ug, dim3(256), 0, s, DEVS(b), t, want_h);
  else
    hipLaunchKernelGGL((k_update_rows<false, double>), ug, dim3(256), 0, s, DEVS(b), t, want_h);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = std::max<int64_t>((int64_t)rn * rn, rn);
  int blocks = (int)std::min<int64_t>(std::max(8, 2048 / b.count), (total + 255) / 256);
  hipLaunchKernelGGL(k_update_sigma, dim3(std::max(blocks, 1), 1, b.count), dim3(256), 0, s, DEVS(b), t,
                     refresh ? 0 : 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (refresh) return launch_gram(b, (t & 1) ^ 1, t + 1, s);
  return hipSuccess;
}

// Last remaining variable: appended without a comparison (Alg. 2).
__device__ __forceinline__ void k_last_body(const Dev& d, int t) {
  const int p = d.p;
  if (rows_left(d, t) != 1 || halted(d.ctl)) return;
  const int32_t* idx = d.idx[t & 1];
  int32_t* order = d.order;
  double* Tall = d.Tall;
  uint8_t* Tstate = d.Tstate;
  double* Terr = d.Terr;
  order[t] = idx[0];
  Tall[(int64_t)t * p + idx[0]] = 0.0;
  Tstate[(int64_t)t * p + idx[0]] = 1;
  Terr[(int64_t)t * p + idx[0]] = 0.0;
  d.Terrp[(int64_t)t * p + idx[0]] = 0.0;
}

__global__ void k_last(const Dev* __restrict__ devs, const Dev one, int t) {
  if (devs)
    k_last_body(devs[blockIdx.z], t);
  else
    k_last_body(one, t);
}

hipError_t launch_last(const Batch& b, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_last, dim3(1, 1, b.count), dim3(1), 0, s, DEVS(b), t);
  return hipGetLastError();
}

// Clear the halt raised by an unfinished iteration (not an error) so that
// further threshold rounds can run.
__device__ __forceinline__ void k_resume_body(const Dev& d) {
  Ctl* ctl = d.ctl;
  if (ctl->status == ST_OK) {
    ctl->halt = 0;
    ctl->halt_iter = -1;
    ctl->arrivals = 0;
    ctl->q_next = 0;
  }
}

__global__ void k_resume(const Dev* __restrict__ devs, const Dev one) {
  if (devs)
    k_resume_body(devs[blockIdx.z]);
  else
    k_resume_body(one);
}

hipError_t launch_resume(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_resume, dim3(1, 1, b.count), dim3(1), 0, s, DEVS(b));
  return hipGetLastError();
}

// ============================================================================
// Alg. 1, last step: causal strengths B from the causal order K
// ============================================================================
// Each variable is regressed on every variable before it in K (Sec. 2.3,
// covariance-based least squares along the order).  All regressions come
// from one factorisation: with C the correlation matrix of the input permuted
// into K order and C = L L^T its Cholesky factor, L_unit = L diag(L)^-1 is
// the unit lower triangle of C = L_unit D L_unit^T, and row t of
// I - L_unit^-1 holds the least-squares coefficients of variable K[t] on
// K[0..t) (standardised units; the sample covariances fit exactly, so this is
// the least-squares solution of the data).  They are then rescaled to the
// input's units, b_ij = b~_ij sd_i / sd_j.

// C0 = the correlation matrix of the normalised input rows, from the first
// Gram (G_ij d_i d_j, unit diagonal).
__global__ void k_corr_snapshot(const Dev d) {
  const int p = d.p;
  const double* __restrict__ G = d.Sig[0];
  const double* __restrict__ dsc = d.dsc[0];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)p * p;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / p), j = (int)(e % p);
    d.C0[e] = i == j ? 1.0 : G[e] * (dsc[i] * dsc[j]);
  }
}

hipError_t launch_corr_snapshot(const Dev& d, hipStream_t s) {
  const int64_t pp = (int64_t)d.p * d.p;
  hipLaunchKernelGGL(k_corr_snapshot, dim3((unsigned)std::min<int64_t>(1024, (pp + 255) / 256)), dim3(256), 0, s,
                     d);
  return hipGetLastError();
}

// Column j of the Cholesky factor (left-looking): one wave per row i >= j
// forms sum_{k<j} L_ik L_jk and, redundantly and identically in every wave,
// the pivot C_jj - sum_{k<j} L_jk^2.  A pivot that is not positive (the
// variables before K[j] determine it) is reported as degenerate.
__global__ __launch_bounds__(256) void k_chol_col(const Dev d, int j) {
  const int p = d.p;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int i = j + blockIdx.x * 4 + wave;
  if (i >= p || halted(d.ctl)) return;
  const int32_t* __restrict__ K = d.order;
  const double* __restrict__ C = d.C0;
  double* __restrict__ L = d.Lch;
  const double* Lj = L + (int64_t)j * p;
  const double* Li = L + (int64_t)i * p;
  double sjj = 0.0, sij = 0.0;
  for (int k = lane; k < j; k += 64) {
    const double ljk = Lj[k];
    sjj += ljk * ljk;
    sij += Li[k] * ljk;
  }
  sjj = wave_sum(sjj);
  sij = wave_sum(sij);
  const double piv = C[(int64_t)K[j] * p + K[j]] - sjj;
  if (!(piv > DEGEN_EPS)) {
    if (i == j && lane == 0) raise_error(d.ctl, ST_DEGENERATE, K[j], -1);
    return;
  }
  const double ljj = sqrt(piv);
  if (lane == 0) L[(int64_t)i * p + j] = i == j ? ljj : (C[(int64_t)K[i] * p + K[j]] - sij) / ljj;
}

// Column j of B_K = I - L_unit^-1 by forward substitution, one work-group:
// m_j = 1 and m_i = -sum_{k=j}^{i-1} (L_ik / L_kk) m_k, written in the
// input's indices and units as B[K[i]][K[j]] = -m_i sd_K[i] / sd_K[j]
// (w_k = m_k / L_kk is kept in LDS).
__global__ __launch_bounds__(256) void k_unit_inverse_col(const Dev d) {
  const int p = d.p, j = blockIdx.x;
  if (j >= p || halted(d.ctl)) return;
  extern __shared__ double w[];
  __shared__ double sh[4];
  const int32_t* __restrict__ K = d.order;
  const double* __restrict__ L = d.Lch;
  double* __restrict__ B = d.Bout;
  if (threadIdx.x == 0) w[0] = 1.0 / L[(int64_t)j * p + j];
  __syncthreads();
  const double sd_j = sqrt(d.stats[2 * K[j] + 1]);
  for (int i = j + 1; i < p; ++i) {
    const double* Li = L + (int64_t)i * p;
    double s = 0.0;
    for (int k = j + threadIdx.x; k < i; k += 256) s += Li[k] * w[k - j];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) {
      w[i - j] = -s / Li[i];
      B[(int64_t)K[i] * p + K[j]] = s * sqrt(d.stats[2 * K[i] + 1]) / sd_j;
    }
    __syncthreads();
  }
}

hipError_t launch_estimate_B(const Dev& d, hipStream_t s) {
  const int p = d.p;
  hipError_t e = launch_fill(d.Bout, (int64_t)p * p, 0.0, s);
  if (e != hipSuccess) return e;
  for (int j = 0; j < p; ++j) {
    hipLaunchKernelGGL(k_chol_col, dim3((p - j + 3) / 4), dim3(256), 0, s, d, j);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_unit_inverse_col, dim3(p), dim3(256), sizeof(double) * p, s, d);
  return hipGetLastError();
}

// ============================================================================
// Self-check of the hardware binary32 exp2 / log2 that the mixed-precision
// rounding bound assumes
// ============================================================================
// Every binary32 argument of the two ranges the per-sample terms use is
// evaluated with the hardware instruction and with the binary64 library
// function (about 2^-52 relative, so its own error is negligible at binary32
// scale): v_exp_f32 over x in [-126, 0] (normal results; below, the term is
// under 2^-126 absolutely) as a relative error, v_log_f32 over [1, 2] as an
// absolute error, both in units of u32 = 2^-24.  Per range: the largest
// error, the sum of signed errors (for the mean), and per binade of the
// argument the sum of signed errors (to bound a systematic bias that a
// data set concentrated in one binade would see).
// Bit patterns are taken in aligned chunks of 2^16 (never across a binade:
// a binade holds 2^23), one chunk per work-group at a time.
constexpr uint32_t SWEEP_CHUNK = 1u << 16;

__global__ __launch_bounds__(256) void k_term_sweep(TermSweep* out, int which, uint32_t lo, uint32_t hi) {
  __shared__ double sh_max[256], sh_sum[256];
  for (uint64_t c0 = (uint64_t)lo + (uint64_t)blockIdx.x * SWEEP_CHUNK; c0 <= hi;
       c0 += (uint64_t)gridDim.x * SWEEP_CHUNK) {
    const uint64_t c1 = min((uint64_t)hi, c0 + SWEEP_CHUNK - 1);
    double mx = 0.0, sm = 0.0;
    for (uint64_t b = c0 + threadIdx.x; b <= c1; b += 256) {
      const float a = __uint_as_float((uint32_t)b);
      double err;
      if (which == 0) {
        const float x = -a;                         // [-126, 0]
        const double ref = exp2((double)x);
        err = ((double)__builtin_amdgcn_exp2f(x) - ref) / ref * 16777216.0;
      } else {
        const double ref = log2((double)a);         // [1, 2]
        err = ((double)__builtin_amdgcn_logf(a) - ref) * 16777216.0;
      }
      mx = fmax(mx, fabs(err));
      sm += err;
    }
    sh_max[threadIdx.x] = mx;
    sh_sum[threadIdx.x] = sm;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        sh_max[threadIdx.x] = fmax(sh_max[threadIdx.x], sh_max[threadIdx.x + s]);
        sh_sum[threadIdx.x] += sh_sum[threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      atomicMax(&out->max_bits[which], (unsigned long long)__double_as_longlong(sh_max[0]));
      atomicAdd(&out->sum[which], sh_sum[0]);
      const int binade = which == 0 ? (int)((c0 >> 23) & 0xff) : 0;   // exponent field of |x|
      if (binade < 160) atomicAdd(&out->binade_sum[which][binade], sh_sum[0]);
    }
    __syncthreads();
  }
}

hipError_t launch_term_sweep(TermSweep* out, hipStream_t s) {
  const uint32_t exp_hi = 0x42FC0000u;   // 126.0f
  const uint32_t log_lo = 0x3F800000u, log_hi = 0x40000000u;   // 1.0f, 2.0f
  hipLaunchKernelGGL(k_term_sweep, dim3(2048), dim3(256), 0, s, out, 0, 0u, exp_hi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_term_sweep, dim3(128), dim3(256), 0, s, out, 1, log_lo, log_hi);
  return hipGetLastError();
}

__global__ void k_fill(double* p, int64_t count, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}
__global__ void k_fill_u8(uint8_t* p, int64_t count, uint8_t v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>(4096, (count + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t* p, int64_t count, uint8_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>(4096, (count + 255) / 256);
  hipLaunchKernelGGL(k_fill_u8, dim3(blocks), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

}  // namespace lingam
