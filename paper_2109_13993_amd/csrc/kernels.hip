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
//                  per-variable terms of Eq. (Itest), computed once per iteration).
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
//   k_update_*     UpdateData and UpdateCovMat (Sec. 3.4): rank-1 update of the
//                  remaining rows and of Sigma, compacting out the root.
#include "lingam_internal.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace lingam {

namespace {

// Eq. (HApp) constants as printed; H(nu) = (1 + log 2 pi) / 2.
constexpr double K1 = 79.047;
constexpr double K2 = 7.4129;
constexpr double BETA = 0.37457;
constexpr double HNU = 1.4189385332046727418;
constexpr double LN2 = 0.69314718055994530942;
constexpr float LOG2E_F = 1.44269504088896340736f;

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
__device__ __forceinline__ void terms_f64(double u, double& lc, double& g) {
  const double a = fabs(u);
  lc += a + log1p(exp(-2.0 * a));
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
template <typename T, int LAYOUT>
__global__ __launch_bounds__(256) void k_standardize(const T* __restrict__ X, int64_t n, int p,
                                                     double* __restrict__ Z, int64_t ldz,
                                                     Ctl* ctl, double* stats) {
  __shared__ double sh[4];
  __shared__ int shi[4];
  const int i = blockIdx.x;
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
  double* z = Z + (int64_t)i * ldz;
  for (int64_t k = threadIdx.x; k < ldz; k += 256) z[k] = k < n ? (load(k) - mean) / sd : 0.0;
  if (threadIdx.x == 0 && stats) {
    stats[2 * i] = mean;
    stats[2 * i + 1] = var;
  }
}

hipError_t launch_standardize(const void* X, int x_dtype, int layout, int64_t n, int p,
                              const Dev& d, hipStream_t s) {
  dim3 g(p), b(256);
  if (x_dtype == 0 && layout == 0)
    hipLaunchKernelGGL((k_standardize<double, 0>), g, b, 0, s, (const double*)X, n, p, d.Z[0], d.ldz, d.ctl, d.stats);
  else if (x_dtype == 0)
    hipLaunchKernelGGL((k_standardize<double, 1>), g, b, 0, s, (const double*)X, n, p, d.Z[0], d.ldz, d.ctl, d.stats);
  else if (layout == 0)
    hipLaunchKernelGGL((k_standardize<float, 0>), g, b, 0, s, (const float*)X, n, p, d.Z[0], d.ldz, d.ctl, d.stats);
  else
    hipLaunchKernelGGL((k_standardize<float, 1>), g, b, 0, s, (const float*)X, n, p, d.Z[0], d.ldz, d.ctl, d.stats);
  return hipGetLastError();
}

// ============================================================================
// a2: CalculateCovMat / refresh -- Sigma = Z Z^T / (n-1) on the FP64 matrix cores
// ============================================================================
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int GT = 32;   // output tile (GT x GT) per work-group, 4 waves of 16 x 16
constexpr int GK = 64;   // samples per LDS stage

__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ Z, int64_t ldz, int64_t n,
                                              int r, double* __restrict__ Sig, int ldsig,
                                              double* __restrict__ dsc, const Ctl* ctl) {
  if (halted(ctl)) return;
  __shared__ double As[GT][GK + 1];
  __shared__ double Bs[GT][GK + 1];
  // upper-triangular tile (ti <= tj) from the linear block index
  const int nt = (r + GT - 1) / GT;
  int ti = 0, rem = blockIdx.x;
  while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
  const int tj = ti + rem;
  const int i0 = ti * GT, j0 = tj * GT;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wy = wave >> 1, wx = wave & 1;
  // each LDS stage is summed by the matrix cores into a fresh accumulator and
  // then added into a Kahan-compensated total, so the rounding error of the
  // n-term dot products stays at the level of one stage
  dbl4 tot = {0.0, 0.0, 0.0, 0.0}, comp = {0.0, 0.0, 0.0, 0.0};
  const int64_t kmax = (n + GK - 1) / GK * GK;  // <= ldz (zero padded)
  for (int64_t k0 = 0; k0 < kmax; k0 += GK) {
    // 32 rows x 64 samples per matrix: 8 doubles per thread
#pragma unroll
    for (int e = 0; e < (GT * GK) / 256; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int row = idx / GK, col = idx % GK;
      const int ra = i0 + row, rb = j0 + row;
      As[row][col] = ra < r ? Z[(int64_t)ra * ldz + k0 + col] : 0.0;
      Bs[row][col] = rb < r ? Z[(int64_t)rb * ldz + k0 + col] : 0.0;
    }
    __syncthreads();
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
  const double inv = 1.0 / (double)(n - 1);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gi = i0 + wy * 16 + (lane >> 4) + 4 * v;
    const int gj = j0 + wx * 16 + (lane & 15);
    if (gi < r && gj < r && gi <= gj) {
      const double val = tot[v] * inv;
      Sig[(int64_t)gi * ldsig + gj] = val;
      Sig[(int64_t)gj * ldsig + gi] = val;
      if (gi == gj) dsc[gi] = 1.0 / sqrt(val);
    }
  }
}

hipError_t launch_gram(const Dev& d, int buf, int r, hipStream_t s) {
  const int nt = (r + GT - 1) / GT;
  hipLaunchKernelGGL(k_gram, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, d.Z[buf], d.ldz, d.n, r,
                     d.Sig[buf], d.p, d.dsc[buf], d.ctl);
  return hipGetLastError();
}

// ============================================================================
// a3: per-variable entropy H(x_u), Eq. (HApp)
// ============================================================================
template <bool MIXED>
__global__ __launch_bounds__(256) void k_entropy(const double* __restrict__ Z, int64_t ldz, int64_t n,
                                                 const double* __restrict__ dsc,
                                                 double* __restrict__ H, const Ctl* ctl) {
  if (halted(ctl)) return;
  __shared__ double sh[4];
  const double* z = Z + (int64_t)blockIdx.x * ldz;
  const double dz = dsc[blockIdx.x];
  double lc = 0.0, g = 0.0;
  if constexpr (MIXED) {
    const float ca = -2.0f * LOG2E_F, cg = -0.5f * LOG2E_F;
    int64_t k = threadIdx.x;
    while (k < n) {
      float flc = 0.f, fg = 0.f;
      for (int c = 0; c < 32 && k < n; ++c, k += 256) terms_mixed((float)(dz * z[k]), ca, cg, flc, fg);
      lc += (double)flc * LN2;
      g += (double)fg;
    }
  } else {
    for (int64_t k = threadIdx.x; k < n; k += 256) terms_f64(dz * z[k], lc, g);
  }
  lc = block_sum256(lc, sh);
  g = block_sum256(g, sh);
  if (threadIdx.x == 0) H[blockIdx.x] = happ_from_sums(lc, g, (double)n);
}

hipError_t launch_entropy(const Dev& d, int buf, int r, int mixed, hipStream_t s) {
  if (mixed)
    hipLaunchKernelGGL(k_entropy<true>, dim3(r), dim3(256), 0, s, d.Z[buf], d.ldz, d.n, d.dsc[buf], d.H, d.ctl);
  else
    hipLaunchKernelGGL(k_entropy<false>, dim3(r), dim3(256), 0, s, d.Z[buf], d.ldz, d.n, d.dsc[buf], d.H, d.ctl);
  return hipGetLastError();
}

// ============================================================================
// iteration set-up: M = "not evaluated", S = 0, everyone below the threshold
// ============================================================================
__global__ void k_iter_init(double* M, uint8_t* pend, double* S, uint8_t* alive, uint8_t* complete,
                            int r, int p, double gamma0, Ctl* ctl) {
  if (halted(ctl)) return;
  const int64_t total = (int64_t)r * r;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e / r), w = (int)(e % r);
    M[(int64_t)x * p + w] = __builtin_nan("");
    pend[(int64_t)x * p + w] = 0;
  }
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < r; x += gridDim.x * blockDim.x) {
    S[x] = 0.0;
    alive[x] = 1;
    complete[x] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->gamma = gamma0;
    ctl->done = 0;
    ctl->root = -1;
    ctl->round = 0;
    ctl->score_arrive = 0;
  }
}

hipError_t launch_iter_init(const Dev& d, int r, double gamma0, hipStream_t s) {
  const int64_t total = (int64_t)r * r;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_iter_init, dim3(blocks), dim3(256), 0, s, d.M, d.pend, d.S, d.alive,
                     d.complete, r, d.p, gamma0, d.ctl);
  return hipGetLastError();
}

// ============================================================================
// a4/a5: the pair kernel
// ============================================================================
// Oriented tile `t` of a band -> (A, B) block indices.
__device__ __forceinline__ void band_tile(const BandArgs& a, int t, int& A, int& B) {
  int d = a.d0;
  for (;;) {
    const int c = tiles_at_distance(a.nb, d, a.both);
    if (t < c) break;
    t -= c;
    ++d;
  }
  if (d == 0) {
    A = B = t;
  } else if (2 * d < a.nb) {
    const int base = t % a.nb, orient = t / a.nb;
    const int other = (base + d) % a.nb;
    if (a.both) {
      A = orient ? other : base;
      B = orient ? base : other;
    } else {
      A = min(base, other);
      B = max(base, other);
    }
  } else {  // 2d == nb
    const int half = a.nb / 2;
    const int base = t % half, orient = t / half;
    A = orient ? base + d : base;
    B = orient ? base : base + d;
  }
}

// Reduce 32 per-lane values to 32 totals spread over the wave: afterwards
// lane l holds total number (l >> 1) & 31 (both lanes of a pair hold it).
__device__ __forceinline__ double reduce_scatter32(double (&v)[32]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const bool hi = lane & 32;
    const double keep = hi ? v[16 + i] : v[i];
    const double send = hi ? v[i] : v[16 + i];
    v[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool hi = lane & 16;
    const double keep = hi ? v[8 + i] : v[i];
    const double send = hi ? v[i] : v[8 + i];
    v[i] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool hi = lane & 8;
    const double keep = hi ? v[4 + i] : v[i];
    const double send = hi ? v[i] : v[4 + i];
    v[i] = keep + __shfl_xor(send, 8, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool hi = lane & 4;
    const double keep = hi ? v[2 + i] : v[i];
    const double send = hi ? v[i] : v[2 + i];
    v[i] = keep + __shfl_xor(send, 4, 64);
  }
  {
    const bool hi = lane & 2;
    const double keep = hi ? v[1] : v[0];
    const double send = hi ? v[0] : v[1];
    v[0] = keep + __shfl_xor(send, 2, 64);
  }
  return v[0] + __shfl_xor(v[0], 1, 64);
}

template <bool MIXED>
__global__ __launch_bounds__(PAIR_THREADS) void k_pair_band(
    const double* __restrict__ Z, int64_t ldz, int64_t n, const double* __restrict__ Sig,
    const double* __restrict__ dsc, const double* __restrict__ M, const uint8_t* __restrict__ alive, double* __restrict__ P,
    uint8_t* __restrict__ pend, const int32_t* __restrict__ idx, int p, BandArgs a, Ctl* ctl) {
  __shared__ double lds[2 * TB][SUB];
  __shared__ uint32_t s_mask[PAIR_WAVES];
  __shared__ int s_stop;
  // the stop decision is read once and shared, so the whole work-group
  // leaves together even if another work-group raises an error meanwhile
  if (threadIdx.x == 0) s_stop = halted(ctl) || ctl->done;

  const int tile = blockIdx.x % a.ntiles;
  const int chunk = blockIdx.x / a.ntiles;
  int A, B;
  band_tile(a, tile, A, B);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = a.r;
  const int v = A * TB + wave;

  // which of the 8 pairs (v, w in B) this wave must evaluate (wave-uniform)
  uint32_t mask = 0;
  if (v < r && alive[v]) {
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      const int w = B * TB + j;
      if (w >= r || w == v) continue;
      if (!__builtin_isnan(M[(int64_t)v * p + w])) continue;
      const bool w_alive = alive[w] != 0;
      const bool take = !w_alive || (A < B) || (A == B && v < w);
      if (take) mask |= 1u << j;
    }
  }
  if (lane == 0) s_mask[wave] = mask;
  __syncthreads();
  uint32_t any = 0;
#pragma unroll
  for (int w = 0; w < PAIR_WAVES; ++w) any |= s_mask[w];
  if (any == 0 || s_stop) return;  // uniform over the work-group

  // per-pair regression coefficient b = Sigma_vw and scale s = 1/sqrt(1 - b^2)
  double bj[TB], sj[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    bj[j] = 0.0;
    sj[j] = 1.0;
    if (mask >> j & 1u) {
      const int w = B * TB + j;
      const double b = Sig[(int64_t)v * p + w] * dsc[v] * dsc[w];
      const double om = 1.0 - b * b;
      if (!(om > DEGEN_EPS)) {
        if (lane == 0) raise_error(ctl, ST_DEGENERATE, idx[v], idx[w]);
      } else {
        bj[j] = b;
        sj[j] = 1.0 / sqrt(om);
      }
    }
  }

  const int64_t k0 = (int64_t)chunk * a.chunk;
  const int64_t kend = min(n, k0 + (int64_t)a.chunk);

  // accumulators: [j][0] lc(r_v), [j][1] g(r_v), [j][2] lc(r_w), [j][3] g(r_w)
  using acc_t = typename std::conditional<MIXED, float, double>::type;
  acc_t acc[TB][4];
#pragma unroll
  for (int j = 0; j < TB; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[j][c] = 0;
  float ca[TB], cg[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    ca[j] = (float)(-2.0 * 1.4426950408889634074 * sj[j]);
    cg[j] = (float)(-0.5 * 1.4426950408889634074 * sj[j] * sj[j]);
  }

  for (int64_t ks = k0; ks < kend; ks += SUB) {
    const int cnt = (int)min((int64_t)SUB, kend - ks);
    // stage rows of blocks A and B (16 x SUB doubles; ldz is a multiple of SUB)
#pragma unroll
    for (int e = 0; e < (2 * TB * SUB / 2) / PAIR_THREADS; ++e) {
      const int idx = threadIdx.x + PAIR_THREADS * e;
      const int row = idx / (SUB / 2), c2 = idx % (SUB / 2);
      const int var = row < TB ? A * TB + row : B * TB + (row - TB);
      double2 val = make_double2(0.0, 0.0);
      if (var < r) {
        val = *reinterpret_cast<const double2*>(Z + (int64_t)var * ldz + ks + 2 * c2);
        const double dv = dsc[var];
        val.x *= dv;
        val.y *= dv;
      }
      *reinterpret_cast<double2*>(&lds[row][2 * c2]) = val;
    }
    __syncthreads();
    if (mask) {
      for (int i = 0; i < SUB / 64; ++i) {
        const int k = i * 64 + lane;
        if (k < cnt) {
          const double zv = lds[wave][k];
#pragma unroll
          for (int j = 0; j < TB; ++j) {
            const double zw = lds[TB + j][k];
            const double rv = __builtin_fma(-bj[j], zw, zv);  // r_v^(w) / s
            const double rw = __builtin_fma(-bj[j], zv, zw);  // r_w^(v) / s
            if constexpr (MIXED) {
              terms_mixed((float)rv, ca[j], cg[j], acc[j][0], acc[j][1]);
              terms_mixed((float)rw, ca[j], cg[j], acc[j][2], acc[j][3]);
            } else {
              double t0 = acc[j][0], t1 = acc[j][1], t2 = acc[j][2], t3 = acc[j][3];
              terms_f64(sj[j] * rv, t0, t1);
              terms_f64(sj[j] * rw, t2, t3);
              acc[j][0] = t0; acc[j][1] = t1; acc[j][2] = t2; acc[j][3] = t3;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (!mask) return;

  // convert to sum(log cosh u + ln 2) and sum(u exp(-u^2/2)), reduce over the wave
  double vals[32];
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    if constexpr (MIXED) {
      vals[4 * j + 0] = (double)acc[j][0] * LN2;
      vals[4 * j + 1] = (double)acc[j][1] * sj[j];
      vals[4 * j + 2] = (double)acc[j][2] * LN2;
      vals[4 * j + 3] = (double)acc[j][3] * sj[j];
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) vals[4 * j + c] = (double)acc[j][c];
    }
  }
  const double tot = reduce_scatter32(vals);
  if ((lane & 1) == 0) {
    const int q = lane >> 1, j = q >> 2, c = q & 3;
    if (mask >> j & 1u) {
      const int w = B * TB + j;
      P[(((int64_t)chunk * p + v) * p + w) * 4 + c] = tot;
      P[(((int64_t)chunk * p + w) * p + v) * 4 + ((c + 2) & 3)] = tot;
    }
  }
  if (chunk == 0 && lane < TB && (mask >> lane & 1u)) {
    const int w = B * TB + lane;
    pend[(int64_t)v * p + w] = 1;
    pend[(int64_t)w * p + v] = 1;
  }
  if (chunk == 0 && lane == 0) {
    atomicAdd(&ctl->pairs_evaluated, (unsigned long long)__popc(mask));
    atomicAdd(&ctl->pairs_computed, (unsigned long long)TB);
  }
}

hipError_t launch_pair_band(const Dev& d, int buf, const BandArgs& a, int mixed, hipStream_t s) {
  dim3 g((unsigned)a.ntiles * (unsigned)a.nchunk), b(PAIR_THREADS);
  if (mixed)
    hipLaunchKernelGGL(k_pair_band<true>, g, b, 0, s, d.Z[buf], d.ldz, d.n, d.Sig[buf], d.dsc[buf], d.M, d.alive,
                       d.P, d.pend, d.idx[buf], d.p, a, d.ctl);
  else
    hipLaunchKernelGGL(k_pair_band<false>, g, b, 0, s, d.Z[buf], d.ldz, d.n, d.Sig[buf], d.dsc[buf], d.M, d.alive,
                       d.P, d.pend, d.idx[buf], d.p, a, d.ctl);
  return hipGetLastError();
}

// ============================================================================
// a5/a6: tests, scores, threshold state, termination and root
// ============================================================================
__global__ __launch_bounds__(256) void k_score(double* __restrict__ M, uint8_t* __restrict__ pend,
                                               const double* __restrict__ P, const double* __restrict__ H,
                                               double* __restrict__ S, uint8_t* __restrict__ alive,
                                               uint8_t* __restrict__ complete, int r, int p, int nchunk,
                                               double n, int round_end, int t, double gamma_mult,
                                               const int32_t* __restrict__ forced, int forced_len,
                                               const int32_t* __restrict__ idx, Ctl* ctl) {
  if (halted(ctl) || ctl->done) return;
  __shared__ int s_last;
  __shared__ double sh_d[256];
  __shared__ int sh_i[256];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int x = blockIdx.x * 4 + wave;
  if (x < r) {
    double s = 0.0;
    int incomplete = 0;
    const double hx = H[x];
    for (int w = lane; w < r; w += 64) {
      if (w == x) continue;
      double m;
      if (pend[(int64_t)x * p + w]) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int c = 0; c < nchunk; ++c) {
          const double* q = P + (((int64_t)c * p + x) * p + w) * 4;
          a0 += q[0]; a1 += q[1]; a2 += q[2]; a3 += q[3];
        }
        const double h_rx = happ_from_sums(a0, a1, n);  // H(r_x^(w))
        const double h_rw = happ_from_sums(a2, a3, n);  // H(r_w^(x))
        m = (H[w] + h_rx) - (hx + h_rw);                // Eq. (Itest)
        M[(int64_t)x * p + w] = m;
        pend[(int64_t)x * p + w] = 0;
      } else {
        m = M[(int64_t)x * p + w];
      }
      if (__builtin_isnan(m)) {
        incomplete = 1;
      } else {
        const double neg = m < 0.0 ? m : 0.0;
        s += neg * neg;
      }
    }
    s = wave_sum(s);
    incomplete = __any(incomplete) ? 1 : 0;
    if (lane == 0) {
      S[x] = s;
      complete[x] = incomplete ? 0 : 1;
    }
  }
  // last work-group to arrive takes the iteration-level decision
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(&ctl->score_arrive, 1u);
    s_last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  double gamma = ctl->gamma;
  int done = 0, root = -1;
  for (int guard = 0; guard < 4096; ++guard) {
    // termination: some complete score <= gamma, every incomplete score > gamma
    int cand = 0, blocked = 0, all_above = 1;
    for (int y = threadIdx.x; y < r; y += 256) {
      const double sy = S[y];
      const int cy = complete[y];
      if (sy <= gamma) {
        all_above = 0;
        if (cy) cand = 1; else blocked = 1;
      }
    }
    cand = __syncthreads_or(cand);
    blocked = __syncthreads_or(blocked);
    all_above = __syncthreads_and(all_above);
    if (cand && !blocked) { done = 1; break; }
    if (round_end && all_above) { gamma *= gamma_mult; continue; }
    break;
  }
  if (done) {
    // root = argmin S over complete variables, lowest position on ties
    double best = INFINITY;
    int bi = 0x7fffffff;
    for (int y = threadIdx.x; y < r; y += 256) {
      if (!complete[y]) continue;
      const double sy = S[y];
      if (sy < best || (sy == best && y < bi)) { best = sy; bi = y; }
    }
    sh_d[threadIdx.x] = best;
    sh_i[threadIdx.x] = bi;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (threadIdx.x < h) {
        const double o = sh_d[threadIdx.x + h];
        const int oi = sh_i[threadIdx.x + h];
        if (o < sh_d[threadIdx.x] || (o == sh_d[threadIdx.x] && oi < sh_i[threadIdx.x])) {
          sh_d[threadIdx.x] = o;
          sh_i[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    root = sh_i[0];
    if (t < forced_len) {
      // teacher forcing: the root is given; find its position
      __shared__ int s_pos;
      if (threadIdx.x == 0) s_pos = -1;
      __syncthreads();
      for (int y = threadIdx.x; y < r; y += 256)
        if (idx[y] == forced[t]) s_pos = y;
      __syncthreads();
      root = s_pos;
    }
  }
  for (int y = threadIdx.x; y < r; y += 256) alive[y] = S[y] <= gamma ? 1 : 0;
  if (threadIdx.x == 0) {
    ctl->gamma = gamma;
    if (done) {
      if (root < 0) {
        raise_error(ctl, ST_INVALID, -1, -1);
      } else {
        ctl->root = root;
        ctl->done = 1;
      }
    } else if (round_end) {
      ctl->round += 1;
    }
    ctl->bands_total += 1;
    ctl->score_arrive = 0;
  }
}

hipError_t launch_score(const Dev& d, int buf, int r, int nchunk, int round_end, int t,
                        double gamma_mult, hipStream_t s) {
  hipLaunchKernelGGL(k_score, dim3((r + 3) / 4), dim3(256), 0, s, d.M, d.pend, d.P, d.H, d.S,
                     d.alive, d.complete, r, d.p, nchunk, (double)d.n, round_end, t, gamma_mult,
                     d.forced, d.forced_len, d.idx[buf], d.ctl);
  return hipGetLastError();
}

// ============================================================================
// end of an iteration: record K, T, H; flag an iteration that is not finished
// ============================================================================
__global__ __launch_bounds__(256) void k_finish_iter(const int32_t* __restrict__ idx,
                                                     const double* __restrict__ S,
                                                     const uint8_t* __restrict__ complete,
                                                     const double* __restrict__ H, int r, int p, int t,
                                                     int32_t* order, double* Tall, uint8_t* Tstate,
                                                     double* Hall, Ctl* ctl) {
  if (halted(ctl)) return;
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
  }
  if (threadIdx.x == 0) {
    order[t] = idx[ctl->root];
    ctl->rounds_total += (unsigned long long)(ctl->round + 1);
  }
}

hipError_t launch_finish_iter(const Dev& d, int buf, int r, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_iter, dim3(1), dim3(256), 0, s, d.idx[buf], d.S, d.complete, d.H, r,
                     d.p, t, d.order, d.Tall, d.Tstate, d.Hall, d.ctl);
  return hipGetLastError();
}

__global__ void k_record_M(const double* __restrict__ M, const int32_t* __restrict__ idx, int r, int p,
                           double* __restrict__ Mrec, const Ctl* ctl) {
  if (halted(ctl)) return;
  const int64_t total = (int64_t)r * r;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e / r), w = (int)(e % r);
    Mrec[(int64_t)idx[x] * p + idx[w]] = M[(int64_t)x * p + w];
  }
}

hipError_t launch_record_M(const Dev& d, int buf, int r, int t, hipStream_t s) {
  const int64_t total = (int64_t)r * r;
  int blocks = (int)std::min<int64_t>(1024, (total + 255) / 256);
  hipLaunchKernelGGL(k_record_M, dim3(std::max(blocks, 1)), dim3(256), 0, s, d.M, d.idx[buf], r, d.p,
                     d.Mrec + (int64_t)t * d.p * d.p, d.ctl);
  return hipGetLastError();
}

// ============================================================================
// a7: UpdateData and UpdateCovMat (Sec. 3.4), compacting out the root
// ============================================================================
__global__ __launch_bounds__(256) void k_update_rows(const double* __restrict__ Z, double* __restrict__ Zn,
                                                     int64_t ldz, int64_t n, const double* __restrict__ Sig,
                                                     const double* __restrict__ dsc, int p, const Ctl* ctl) {
  if (halted(ctl) || !ctl->done) return;
  const int root = ctl->root;
  const int wn = blockIdx.y;                  // new position
  const int w = wn + (wn >= root ? 1 : 0);    // old position
  const double dw = dsc[w], dr = dsc[root];
  const double b = Sig[(int64_t)w * p + root] * dw * dr;   // correlation of the normalised rows
  const double sc = 1.0 / sqrt(1.0 - b * b);
  const double* zr = Z + (int64_t)root * ldz;
  const double* zw = Z + (int64_t)w * ldz;
  double* zo = Zn + (int64_t)wn * ldz;
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
    zo[k] = (dw * zw[k] - b * (dr * zr[k])) * sc;
}

__global__ __launch_bounds__(256) void k_update_sigma(const double* __restrict__ Sig, double* __restrict__ Sn,
                                                      const double* __restrict__ dsc, double* __restrict__ dscn,
                                                      const int32_t* __restrict__ idx, int32_t* __restrict__ idxn,
                                                      int r, int p, int recursion, const Ctl* ctl) {
  if (halted(ctl) || !ctl->done) return;
  const int root = ctl->root;
  const int rn = r - 1;
  const int64_t total = (int64_t)rn * rn;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid < rn) {
    const int w = (int)gid + ((int)gid >= root ? 1 : 0);
    idxn[gid] = idx[w];
    if (recursion) dscn[gid] = 1.0;  // the recursion's rows are unit-variance by construction
  }
  if (!recursion) return;
  for (int64_t e = gid; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int an = (int)(e / rn), bn = (int)(e % rn);
    const int a = an + (an >= root ? 1 : 0), b = bn + (bn >= root ? 1 : 0);
    double val;
    if (an == bn) {
      val = 1.0;
    } else {
      const double da = dsc[a], db = dsc[b], dr = dsc[root];
      const double ba = Sig[(int64_t)a * p + root] * da * dr, bb = Sig[(int64_t)b * p + root] * db * dr;
      const double bab = Sig[(int64_t)a * p + b] * da * db;
      val = (bab - ba * bb) / (sqrt(1.0 - ba * ba) * sqrt(1.0 - bb * bb));
    }
    Sn[(int64_t)an * p + bn] = val;
  }
}

hipError_t launch_update(const Dev& d, int buf, int r, int refresh, hipStream_t s) {
  const int rn = r - 1;
  if (rn <= 0) return hipSuccess;
  int xblocks = (int)std::min<int64_t>(64, (d.n + 255) / 256);
  hipLaunchKernelGGL(k_update_rows, dim3(xblocks, rn), dim3(256), 0, s, d.Z[buf], d.Z[buf ^ 1], d.ldz,
                     d.n, d.Sig[buf], d.dsc[buf], d.p, d.ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = std::max<int64_t>((int64_t)rn * rn, rn);
  int blocks = (int)std::min<int64_t>(2048, (total + 255) / 256);
  hipLaunchKernelGGL(k_update_sigma, dim3(std::max(blocks, 1)), dim3(256), 0, s, d.Sig[buf], d.Sig[buf ^ 1],
                     d.dsc[buf], d.dsc[buf ^ 1], d.idx[buf], d.idx[buf ^ 1], r, d.p, refresh ? 0 : 1, d.ctl);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (refresh) return launch_gram(d, buf ^ 1, rn, s);
  return hipSuccess;
}

// Last remaining variable: appended without a comparison (Alg. 2, lines 1-3).
__global__ void k_last(const int32_t* idx, int p, int t, int32_t* order, double* Tall, uint8_t* Tstate,
                       const Ctl* ctl) {
  if (halted(ctl)) return;
  order[t] = idx[0];
  Tall[(int64_t)t * p + idx[0]] = 0.0;
  Tstate[(int64_t)t * p + idx[0]] = 1;
}

hipError_t launch_last(const Dev& d, int buf, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_last, dim3(1), dim3(1), 0, s, d.idx[buf], d.p, t, d.order, d.Tall, d.Tstate, d.ctl);
  return hipGetLastError();
}

// Clear the halt raised by an unfinished iteration (not an error) so that
// further threshold rounds can run.
__global__ void k_resume(Ctl* ctl) {
  if (ctl->status == ST_OK) {
    ctl->halt = 0;
    ctl->halt_iter = -1;
  }
}

hipError_t launch_resume(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_resume, dim3(1), dim3(1), 0, s, d.ctl);
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
