// Internal declarations shared by the HIP kernels and the host driver of the
// MI355X DirectLiNGAM causal-order search.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lingam.h"

namespace lingam {

// A fixed block of device memory on the current device that a call carves
// all of its buffers from (no allocation); `who` names the owner in error
// messages.
struct FixedBlock {
  char* base;
  uint64_t cap;
  const char* who;
};
// lingam_fit_order with every device buffer carved from `block` and nothing
// allocated: no device memory, streams or events are created, and the search
// runs on opts->stream (NULL = the null stream).  opts->workspace and
// opts->profile are rejected.  (driver.cpp)
lingam_status fit_order_in_block(const void* X, int64_t n, int64_t p, const lingam_opts* opts,
                                 lingam_result* out, const FixedBlock& block);
// Detail text for lingam_last_error() on the calling thread.  (driver.cpp)
void set_last_error(const char* msg);

// Variables per target block of the pair kernel.
constexpr int TB = 8;
// Row stride unit of the stored data (doubles); every sample range a kernel
// stages starts at a multiple of it.
constexpr int SUB = 256;

// Samples per work-group chunk: at most 32 per lane, so the binary32 lane
// sums of the mixed mode never run over more than 32 terms.
constexpr int CHUNK_DEFAULT = 2048;
constexpr int CHUNK_MAX_MIXED = 2048;
// Degeneracy guard on 1 - corr^2 of an evaluated pair (and row variance).
constexpr double DEGEN_EPS = 1e-12;

// The split Gram (CalculateCovMat and its refreshes): output tiles of GT x GT
// per work-group, GK samples per LDS stage, and a split of the samples into
// slices with enough work-groups to fill the device, each slice at least
// four stages long.
constexpr int GT = 32;
constexpr int GK = 64;
constexpr int gram_slices(int r, int64_t n, int max_slices) {
  const int nt = (r + GT - 1) / GT;
  const int tiles = nt * (nt + 1) / 2;
  int sl = (2048 + tiles - 1) / tiles;
  const int64_t stages = (n + GK - 1) / GK;
  const int64_t cap = stages / 4 > 1 ? stages / 4 : 1;
  if ((int64_t)sl > cap) sl = (int)cap;
  if (sl > max_slices) sl = max_slices;
  return sl < 1 ? 1 : sl;
}
// Rows of partial sums the Gram of r <= p rows needs at most (slices x r),
// over every r: the partial-sum buffer holds this many rows of p.
inline int64_t gram_partial_rows(int64_t p, int64_t n, int max_slices) {
  int64_t most = 0;
  for (int64_t r = 1; r <= p; ++r) {
    const int64_t v = (int64_t)gram_slices((int)r, n, max_slices) * r;
    if (v > most) most = v;
  }
  return most;
}
constexpr int PAIR_SLOTS = 2048;
// Sample segments of a row in the row update (one work-group each); with no
// Gram refresh between two iterations the update also sums the new row's
// entropy terms per segment, and the next iteration only adds them up.
constexpr int ENT_SEGS = 16;

enum Status : int32_t { ST_OK = 0, ST_INVALID = 1, ST_NONFINITE = 2, ST_DEGENERATE = 3 };

// Device-resident control block of one search.  Written only by kernels
// (and zeroed by the host before the first launch).
struct Ctl {
  double gamma;         // current threshold of this iteration
  int32_t done;         // 1 = root of the current iteration found
  int32_t root;         // root position (index into the compacted rows)
  int32_t halt;         // 1 = every later kernel returns at once
  int32_t halt_iter;    // iteration that raised halt (-1 = none)
  int32_t status;       // Status of the first error
  int32_t bad_i, bad_j; // compacted positions (pair error) or original index (row error)
  int32_t round;        // threshold round of the current iteration
  uint32_t arrivals;     // work-groups of the running score launch that have finished
  uint32_t q_next;       // batch queue: pair-kernel items of the band claimed so far
  int32_t n_alive;        // entries of the alive list (incomplete variables with S <= gamma)
  int32_t tb_next;        // target blocks [tb_next, tb_next + ntb_next) of the next band
  int32_t ntb_next;
  int32_t iter_bands;     // bands run in the current iteration
  int32_t win_bands;      // most bands of one iteration since the host last looked
  double last_root_S;     // score of the previous iteration's root (adaptive gamma0)
  unsigned long long rounds_total;
  unsigned long long bands_total;
};

// Device pointers and sizes of one search.  The kernels read it from device
// memory: an array of them, one per data set of a batch, indexed by
// blockIdx.z (a single search is a batch of one).
struct Dev {
  int p = 0;                 // number of variables
  int64_t n = 0;             // samples
  const void* X = nullptr;   // input rows on the device (read by the standardisation only)
  int x_dtype = 0;           // 0 = double, 1 = float
  int layout = 0;            // 0 = p x n (row = variable), 1 = n x p
  int nchunk = 1;            // sample chunks of the pair kernel, ceil(n / chunk)
  int limit = 0;             // iterations to run (p, or fewer when max_roots is set)
  // Pair counters, spread over PAIR_SLOTS addresses (slot = wave % PAIR_SLOTS)
  // so that their atomics do not queue on one address: [0, PAIR_SLOTS)
  // evaluated pairs, [PAIR_SLOTS, 2 PAIR_SLOTS) pairs computed.  Summed by the host.
  unsigned long long* pair_slots = nullptr;
  int messaging = 1;         // 1 = a pair's reverse test is its negation (Sec. 3.1); 0 = each
                             // direction evaluated by its own row (ablation)
  int band_k0 = 4;           // target blocks of an iteration's first band (every block: no threshold)
  int band_adapt = 1;        // 1 = size later bands from the alive count, 0 = band_k0 blocks each
  int64_t ldz = 0;           // row stride of Z (elements), multiple of SUB
  // p x ldz normalised rows (ping-pong by iteration parity), binary64, or
  // binary32 when store32 is set (FP32-storage precision)
  void* Z[2] = {nullptr, nullptr};
  int store32 = 0;
  // Sig holds G, the covariance of the rows the Gram was taken of (ld = p),
  // and dsc the row scales d_i = 1/sqrt(G_ii): the normalised rows are d_i z_i
  // and their correlation is b_ij = G_ij d_i d_j.  The entropy pass at the
  // start of the iteration stores the rows as d_i z_i (in place), so every
  // later kernel of the iteration reads normalised rows and uses d only for
  // b.  Re-normalising from the Gram this way keeps the rank-1 recursion from
  // amplifying rounding in the row variances.
  double* Sig[2] = {nullptr, nullptr};
  double* dsc[2] = {nullptr, nullptr};
  // Positions of the remaining variables.  After each root the survivors
  // are placed in ascending order of their score in the finished iteration
  // (ties by original index), so the next iteration's first target blocks
  // hold the variables most likely to be causes, and its threshold prunes
  // the other rows early.  Every result is formed in an order that does not
  // depend on positions (scores sum their tests in ascending original
  // index, ties go to the lowest original index), so positions change which
  // pairs get evaluated, never a value.
  int32_t* idx[2] = {nullptr, nullptr};   // [p] position -> original index
  int32_t* ord[2] = {nullptr, nullptr};   // [p] rank by original index -> position
  int32_t* perm = nullptr;                // [p] new position -> old position (set at each root)
  double* Hp = nullptr;      // [p][ENT_SEGS][2] entropy sums of the updated rows, per segment
  int mixed = 0;             // 1 = mixed-precision per-sample terms
  double* H = nullptr;       // [p] entropy estimate per compacted row
  double* eH = nullptr;      // [p] rounding bound of H (mixed mode; 0 in FP64 mode)
  double* Meps = nullptr;    // p x p rounding bound of each evaluated test (mixed mode)
  double* eT = nullptr;      // [p] rounding bound of each score (mixed mode)
  double* Terr = nullptr;    // [p*p] eT per iteration, by original index
  // the probable bounds (independent rounding errors, Hoeffding) beside the
  // worst-case ones: per H, per test, per score, per iteration
  double* eHp = nullptr;
  double* Mepsp = nullptr;
  double* eTp = nullptr;
  double* Terrp = nullptr;
  double* M = nullptr;       // p x p test matrix of the iteration (NaN = not evaluated)
  double* S = nullptr;       // [p] scores (sum of min(0, M)^2 over evaluated pairs)
  uint8_t* alive = nullptr;  // [p] S <= gamma and some test not evaluated, at the last decision
  int32_t* alive_list = nullptr;  // [p] positions with alive = 1, ascending
  uint8_t* complete = nullptr;  // [p] every pair of the row evaluated
  uint8_t* pend = nullptr;   // p x p: partial sums written, M not yet formed
  double* P = nullptr;       // [nchunk][p][p][4] per-chunk partial sums
  Ctl* ctl = nullptr;
  int32_t* order = nullptr;  // [p]
  double* Tall = nullptr;    // [p*p]
  uint8_t* Tstate = nullptr; // [p*p]
  double* Hall = nullptr;    // [p*p]
  double* Mrec = nullptr;    // [rec*p*p]
  int rec = 0;
  const int32_t* forced = nullptr;  // device copy of the forced prefix
  int forced_len = 0;
  double* stats = nullptr;   // [2*p] per-row mean/variance of the input (diagnostics)
  double* Gp = nullptr;      // [slices][r][p] per-slice partial Gram (gram_partial_rows x p)
  int gram_slices_max = 1;   // largest sample split of the Gram
  // causal strengths from the order (Alg. 1, last step), when asked for
  double* C0 = nullptr;      // p x p correlation of the normalised input
  double* Lch = nullptr;     // p x p Cholesky factor of C0 in the order's permutation (lower)
  double* Bout = nullptr;    // p x p B in the input's indices and units
};

// Largest p for which B is estimated (one column of the inverse in LDS).
constexpr int B_MAX_P = 8000;

// Samples per pair-kernel band that later bands of round 0 aim at: their
// target-block count is chosen so that (alive rows) x (targets) x n is
// about this, rounded up to whole rounds of the work-groups when it fills
// at least one, between band_k0 and the blocks left.  A single mixed-mode
// search takes larger bands (its per-band overhead weighs more against its
// fast pair kernel): 6e7 up to p = 1000, then growing as (p / 1000)^4 up
// to 1.6e9 (p = 1588: 3.8e8, about 1.4x faster than 6e7 on flux-like
// stand-ins at n = 10000; up to p = 1000 larger bands lost up to 9% on
// strongly pruned searches).  FP64 searches and batches, whose launches
// carry more work per band, take smaller ones.  Chosen by measurement at
// p = 100 ... 2339 and on the batch workloads.
constexpr double BAND_TARGET_SINGLE_MIXED_MIN = 6e7;
constexpr double BAND_TARGET_SINGLE_MIXED_MAX = 1.6e9;
constexpr double BAND_TARGET_DEFAULT = 2e7;
inline double band_target_single_mixed(int p) {
  const double q = (double)p / 1000.0;
  const double t = BAND_TARGET_SINGLE_MIXED_MIN * (q * q) * (q * q);
  return t < BAND_TARGET_SINGLE_MIXED_MIN ? BAND_TARGET_SINGLE_MIXED_MIN
                                          : (t > BAND_TARGET_SINGLE_MIXED_MAX ? BAND_TARGET_SINGLE_MIXED_MAX : t);
}

// Parameters of one band launch of the pair kernel.  Which target blocks
// the band covers is decided on the device (Ctl::tb_next, ntb_next), so
// the host only queues band slots; a slot after the iteration is decided
// returns at once.
struct BandArgs {
  int chunk;      // samples per chunk
  int rows_per_group;  // alive rows per pair-kernel work-group
  int groups;     // pair-kernel work-groups one data set's later bands run on
  double band_target;  // pair-samples a later band of round 0 aims at
  int score_wave_rows = 0;  // score rows of at most this many variables one per wave (else per work-group)
};

// What a launch covers: `count` data sets whose descriptors are at `dd` on
// the device, every one at iteration t (r = p - t variables left).  The
// host-side maxima size the grids; each work-group reads its own sizes.
struct Batch {
  const Dev* dd = nullptr;   // device array [count]
  int count = 1;
  Dev one;                   // the descriptor itself when count == 1
  int p_max = 0;             // largest p of the batch
  int64_t n_max = 0;         // largest n
  int nchunk_max = 1;
  int gram_slices_max = 1;
  int mixed = 0;
  int store32 = 0;           // rows stored in binary32 (every data set of the batch)
  int queue = 1;             // batches: pair work on the device work queue (scores in grid slices)
  // Sets that have an iteration at t: act[0, active_at(t)) on the device;
  // act_until[i] (host, descending) is the first iteration set act[i] no
  // longer has.
  const int32_t* act = nullptr;
  const int* act_until = nullptr;
  int active_at(int t) const {
    int lo = 0, hi = count;   // act_until is descending: count the entries > t
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (act_until[mid] > t) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
};

// ---- launch wrappers (kernels.hip) --------------------------------------
// t is the iteration every data set of the batch is at; buf = t & 1 selects
// the ping-pong buffers.
hipError_t launch_standardize(const Batch& b, hipStream_t s);
hipError_t launch_gram(const Batch& b, int buf, int t, hipStream_t s);
// Start of iteration t: the entropies of the remaining rows and the
// iteration's set-up (tests not evaluated, scores 0, threshold state).
// fused: the row update of iteration t - 1 left the entropy sums (no Gram
// refresh in between), so only their segments are added up.
hipError_t launch_iter_start(const Batch& b, int t, double gamma0, double adapt, int threshold, int fused,
                             hipStream_t s);
// Shape of the later (bounded) pair-kernel bands of a launch over b: rows
// per work-group and the work-groups one data set gets.
void pair_band_shape(const Batch& b, int& rows_per_group, int& groups);
// ev0/ev1 (optional): events that take the start and end time of the launch
// itself (nullptr: an untimed launch).
hipError_t launch_pair_band(const Batch& b, int t, const BandArgs& a, int dense, int ntb_hint, hipStream_t s,
                            hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// The tests of iteration t by one of the baseline mappings (lingam_pair_strategy 1-3):
// FP64 single searches, every ordered pair, chunk partials of `chunk` samples.
hipError_t launch_pair_baseline(const Batch& b, int t, int strategy, int chunk, hipStream_t s);
hipError_t launch_score(const Batch& b, int t, const BandArgs& a, double gamma_mult, int dense, int ntb_hint,
                        hipStream_t s);
hipError_t launch_window_reset(const Batch& b, hipStream_t s);
hipError_t launch_record_M(const Batch& b, int t, hipStream_t s);
// End of iteration t: its results (order, T, H, bounds; an unfinished
// iteration halts instead), UpdateData and UpdateCovMat, and with refresh
// the Gram of the updated rows.
hipError_t launch_iter_end(const Batch& b, int t, int refresh, hipStream_t s);
hipError_t launch_last(const Batch& b, int t, hipStream_t s);
hipError_t launch_resume(const Batch& b, hipStream_t s);
hipError_t launch_gather(const double* X, int64_t n_src, int64_t p, const int64_t* idx, int64_t n_idx,
                         double* out, hipStream_t s);
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s);
// Initial contents of every data set's buffers and control block (after the
// descriptors are on the device; before the first kernel of the search).
hipError_t launch_init_sets(const Batch& b, hipStream_t s);
// The pair counters of every data set summed into pair_slots[0] (pairs
// evaluated) and [1] (computed), after the search.
hipError_t launch_sum_slots(const Batch& b, hipStream_t s);
// Hardware binary32 exp2 / log2 against binary64 over every argument of the
// ranges the mixed-precision terms use (errors in units of u32 = 2^-24):
// [0] v_exp_f32 on [-126, 0] (relative), [1] v_log_f32 on [1, 2] (absolute).
struct TermSweep {
  unsigned long long max_bits[2];  // largest |error| (bit pattern of a non-negative double)
  double sum[2];                   // sum of signed errors
  double binade_sum[2][160];       // exp2: per exponent field of |x|; log2: [0] only
};
hipError_t launch_term_sweep(TermSweep* out, hipStream_t s);
// C0 from the first Gram (after launch_gram at t = 0).
hipError_t launch_corr_snapshot(const Dev& d, hipStream_t s);
// B from C0 and the causal order in d.order (host-side descriptor d).
hipError_t launch_estimate_B(const Dev& d, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t count, uint8_t v, hipStream_t s);

}  // namespace lingam
