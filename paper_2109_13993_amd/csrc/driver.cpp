// Host runtime and C ABI of the MI355X DirectLiNGAM causal-order search.
//
// One call of lingam_fit_order runs Alg. 3 of ParaLiNGAM (arXiv 2109.13993)
// on one GPU: NormalizeData and CalculateCovMat once, then for every
// iteration the per-variable entropies, the threshold rounds of
// ParaFindRoot (pair kernel + score kernel, Sec. 3.2-3.3 and 4.3), and the
// UpdateData / UpdateCovMat rank-1 updates (Sec. 3.4).  Every decision of an
// iteration (threshold, termination, root) is taken on the device, so the
// host only queues launches; it synchronises once every SYNC_EVERY
// iterations to check for errors and for iterations that needed more
// threshold rounds than were queued.
//
// lingam_fit_order_batch runs many independent searches through the same
// kernels: every launch covers all data sets of the batch (one descriptor
// each, grid dimension z), each at the same iteration.  A data set whose
// iteration needs more threshold rounds than were queued sits out the rest
// of the batch and is finished on its own afterwards.
#include "lingam.h"
#include "lingam_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

using namespace lingam;

namespace {

thread_local std::string g_last_error;

struct HipFail {
  hipError_t err;
  const char* what;
  int line;
};

#define HIPCHK(x)                                         \
  do {                                                    \
    hipError_t e_ = (x);                                  \
    if (e_ != hipSuccess) throw HipFail{e_, #x, __LINE__}; \
  } while (0)

struct NoMem {
  uint64_t need, have;
};

// Device memory of one call, carved out of one block: the caller's
// workspace, the no-allocation entry point's static device array, or one
// hipMalloc of the whole size.  A sizing pass (base == nullptr) runs the same
// sequence of get() calls and only counts bytes, so the size a call needs
// and the layout it uses come from one piece of code.  Every buffer starts
// on a 256-byte boundary.
struct Arena {
  char* base = nullptr;
  uint64_t off = 0, cap = 0;
  template <class T>
  T* get(size_t count) {
    if (count == 0) count = 1;
    off = (off + 255) & ~(uint64_t)255;
    const uint64_t at = off;
    off += (uint64_t)count * sizeof(T);
    if (!base) return nullptr;
    if (off > cap) throw NoMem{off, cap};
    return reinterpret_cast<T*>(base + at);
  }
};

// One hipMalloc of a call's whole workspace, released on every exit path.
struct OwnedMem {
  void* p = nullptr;
  ~OwnedMem() {
    if (p) (void)hipFree(p);
  }
};

// Restores the calling thread's current device on every exit path.
struct DeviceGuard {
  int prev = -1;
  void set(int dev) {
    if (dev < 0) return;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) cur = -1;
    if (cur == dev) return;
    prev = cur;
    if (hipSetDevice(dev) != hipSuccess) throw HipFail{hipErrorInvalidDevice, "hipSetDevice", __LINE__};
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

struct OwnedStream {
  hipStream_t s = nullptr;
  bool owned = false;
  ~OwnedStream() {
    if (owned && s) (void)hipStreamDestroy(s);
  }
};

constexpr int SYNC_EVERY = 16;   // iterations queued between host checks
constexpr int QUEUED_ROUNDS = 4; // threshold rounds queued per iteration
constexpr int GRAM_SLICES_MAX = 16;  // sample slices of the split Gram
// Target blocks of an iteration's first threshold band.  Its targets are
// the variables that scored best in the previous iteration, and for a single
// mixed-mode search a wider first band (4 blocks) kills most rows at once;
// FP64 searches and batches, whose per-band overhead weighs less, do best
// with one block.  Chosen by measurement (1 to 10 blocks tried).
constexpr int BAND_BLOCKS_DEFAULT = 1;
constexpr int BAND_BLOCKS_SINGLE_MIXED = 4;
constexpr double GAMMA_ADAPT = 1.5;  // adaptive gamma0 = this x previous root score (by measurement)
// Default Gram refresh period of the mixed mode: between refreshes the
// paper's rank-1 UpdateCovMat carries the covariance; its drift over a few
// iterations stays far below the binary32 rounding of the per-sample terms.
constexpr int REFRESH_MIXED = 16;

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct Plan {
  int chunk = CHUNK_DEFAULT;
  int nchunk = 1;
  int band_blocks = 4;   // target blocks (of 8 variables) per threshold band
};

Plan make_plan(int64_t n, const lingam_opts& o, bool single) {
  Plan pl;
  int chunk = o.chunk_samples > 0 ? o.chunk_samples : CHUNK_DEFAULT;
  if (o.precision != LINGAM_PREC_FP64) chunk = std::min(chunk, CHUNK_MAX_MIXED);
  pl.chunk = chunk;
  pl.nchunk = (int)((n + chunk - 1) / chunk);
  pl.band_blocks = o.band_blocks > 0 ? o.band_blocks
                 : o.first_band_blocks > 0 ? o.first_band_blocks
                 : (single && o.precision != LINGAM_PREC_FP64 ? BAND_BLOCKS_SINGLE_MIXED : BAND_BLOCKS_DEFAULT);
  return pl;
}

// Band slots of an iteration at which the largest data set has r variables:
// at most the round-0 bands of band_k0 blocks each, plus QUEUED_ROUNDS - 1
// full-band rounds.  (The device picks each slot's blocks; unused slots
// return at once.)
int max_slots(int r, int k0) {
  const int nb = (r + TB - 1) / TB;
  return (nb + k0 - 1) / k0 + QUEUED_ROUNDS - 1;
}

lingam_status fail(lingam_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

lingam_status validate_opts(const lingam_opts& o) {
  if (o.struct_size != sizeof(lingam_opts)) return fail(LINGAM_E_INVALID, "opts.struct_size mismatch");
  if (o.precision != LINGAM_PREC_FP64 && o.precision != LINGAM_PREC_MIXED &&
      o.precision != LINGAM_PREC_FP32_STORAGE)
    return fail(LINGAM_E_INVALID, "unknown precision");
  if (o.layout != LINGAM_LAYOUT_VAR_MAJOR && o.layout != LINGAM_LAYOUT_SAMPLE_MAJOR)
    return fail(LINGAM_E_INVALID, "unknown layout");
  if (o.x_dtype != 0 && o.x_dtype != 1) return fail(LINGAM_E_INVALID, "x_dtype must be 0 or 1");
  if (o.max_roots < 0) return fail(LINGAM_E_INVALID, "max_roots < 0");
  if (o.chunk_samples < 0 || o.chunk_samples % SUB != 0)
    return fail(LINGAM_E_INVALID, "chunk_samples must be a multiple of 256");
  if (o.band_blocks < 0) return fail(LINGAM_E_INVALID, "band_blocks < 0");
  if (o.first_band_blocks < 0) return fail(LINGAM_E_INVALID, "first_band_blocks < 0");
  if (o.messaging != 0 && o.messaging != 1) return fail(LINGAM_E_INVALID, "messaging must be 0 or 1");
  if (o.pair_strategy < LINGAM_PAIR_DEFAULT || o.pair_strategy > LINGAM_PAIR_BLOCK_COMPARE)
    return fail(LINGAM_E_INVALID, "unknown pair_strategy");
  if (o.pair_strategy != LINGAM_PAIR_DEFAULT &&
      (o.precision != LINGAM_PREC_FP64 || o.use_threshold || o.messaging))
    return fail(LINGAM_E_INVALID, "a baseline pair_strategy needs FP64, use_threshold = 0 and messaging = 0");
  if (o.record_M_iters < 0) return fail(LINGAM_E_INVALID, "record_M_iters < 0");
  if (o.estimate_B != 0 && o.estimate_B != 1) return fail(LINGAM_E_INVALID, "estimate_B must be 0 or 1");
  if (o.batch_queue != 0 && o.batch_queue != 1) return fail(LINGAM_E_INVALID, "batch_queue must be 0 or 1");
  if (o.graph != 0 && o.graph != 1) return fail(LINGAM_E_INVALID, "graph must be 0 or 1");
  if (!(o.band_target >= 0.0) || o.band_target > 1e15) return fail(LINGAM_E_INVALID, "band_target out of range");
  if (o.forced_len < 0 || (o.forced_len > 0 && !o.forced_order))
    return fail(LINGAM_E_INVALID, "bad forced_order / forced_len");
  return LINGAM_OK;
}

lingam_status validate_shape(int64_t n, int64_t p) {
  if (n < 2) return fail(LINGAM_E_INVALID, "n must be >= 2");
  if (p < 1) return fail(LINGAM_E_INVALID, "p must be >= 1");
  if (p > 65535) return fail(LINGAM_E_INVALID, "p must be <= 65535");
  if (n > ((int64_t)1 << 40) || p * n > ((int64_t)1 << 40)) return fail(LINGAM_E_INVALID, "p * n too large");
  return LINGAM_OK;
}

lingam_status validate(const void* X, int64_t n, int64_t p, const lingam_opts& o, const lingam_result* out) {
  if (!X) return fail(LINGAM_E_INVALID, "X is NULL");
  if (!out || !out->order) return fail(LINGAM_E_INVALID, "result or result->order is NULL");
  lingam_status st = validate_opts(o);
  if (st != LINGAM_OK) return st;
  st = validate_shape(n, p);
  if (st != LINGAM_OK) return st;
  if (o.record_M_iters > p) return fail(LINGAM_E_INVALID, "record_M_iters out of range");
  if (o.record_M_iters > 0 && !out->M) return fail(LINGAM_E_INVALID, "record_M_iters > 0 but result->M is NULL");
  if (o.estimate_B) {
    if (!out->B) return fail(LINGAM_E_INVALID, "estimate_B set but result->B is NULL");
    if (o.max_roots > 0 && o.max_roots < p) return fail(LINGAM_E_INVALID, "estimate_B needs the full order");
    if (p > B_MAX_P) return fail(LINGAM_E_INVALID, "estimate_B supports p <= 8000");
  }
  if (o.forced_len > p) return fail(LINGAM_E_INVALID, "bad forced_order / forced_len");
  if (o.forced_len > 0) {
    std::vector<char> seen((size_t)p, 0);
    for (int k = 0; k < o.forced_len; ++k) {
      const int32_t v = o.forced_order[k];
      if (v < 0 || v >= p || seen[(size_t)v]) return fail(LINGAM_E_INVALID, "forced_order is not a prefix of a permutation");
      seen[(size_t)v] = 1;
    }
  }
  return LINGAM_OK;
}

void reset_result(lingam_result* out, int64_t p, int rec) {
  for (int64_t t = 0; t < p; ++t) out->order[t] = -1;
  if (out->T) for (int64_t k = 0; k < p * p; ++k) out->T[k] = NAN;
  if (out->T_state) std::memset(out->T_state, 0, (size_t)(p * p));
  if (out->H) for (int64_t k = 0; k < p * p; ++k) out->H[k] = NAN;
  if (out->M) for (int64_t k = 0; k < (int64_t)rec * p * p; ++k) out->M[k] = NAN;
  if (out->T_err_bound) for (int64_t k = 0; k < p * p; ++k) out->T_err_bound[k] = NAN;
  if (out->B) for (int64_t k = 0; k < p * p; ++k) out->B[k] = NAN;
  if (out->T_err_prob) for (int64_t k = 0; k < p * p; ++k) out->T_err_prob[k] = NAN;
  out->pairs_evaluated = out->pair_samples = out->pairs_computed = 0;
  out->threshold_rounds = out->bands = 0;
  out->seconds_total = out->seconds_device = out->seconds_pair_kernel = 0.0;
  out->pair_kernel_launches = 0;
  out->iterations = 0;
  out->bad_i = out->bad_j = -1;
  out->status = LINGAM_OK;
}

// Optional timing of the pair-kernel launches: a pair of events that take
// each launch's own start and end time on its stream, summed at the end of
// the call.
struct PairTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  uint64_t launches = 0;
  ~PairTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  hipEvent_t next() {
    if (used == ev.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      ev.push_back(e);
    }
    return ev[used++];
  }
  double total_seconds() {
    double s = 0.0;
    for (size_t k = 0; k + 1 < used; k += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) s += ms * 1e-3;
    }
    return s;
  }
};

// Buffers of one data set (device memory from `al`), its iteration limit
// and host-side shape.
struct SetInfo {
  int64_t p = 0, n = 0;
  int limit = 0;        // iterations to run (p, or max_roots)
  Ctl* ctl = nullptr;   // its control block inside the call's Ctl array
};

Dev carve_set(Arena& al, int64_t n, int64_t p, const Plan& pl, const lingam_opts& o, bool mixed, Ctl* ctl) {
  Dev d;
  d.p = (int)p;
  d.n = n;
  d.ldz = round_up(n, SUB);
  d.nchunk = (int)((n + pl.chunk - 1) / pl.chunk);
  d.mixed = mixed ? 1 : 0;
  d.store32 = o.precision == LINGAM_PREC_FP32_STORAGE ? 1 : 0;
  d.x_dtype = o.x_dtype;
  d.layout = o.layout;
  const size_t P = (size_t)p, pp = P * P;
  const size_t zbytes = P * (size_t)d.ldz * (d.store32 ? sizeof(float) : sizeof(double));
  d.Z[0] = al.get<uint8_t>(zbytes);
  d.Z[1] = al.get<uint8_t>(zbytes);
  d.Sig[0] = al.get<double>(pp);
  d.Sig[1] = al.get<double>(pp);
  d.dsc[0] = al.get<double>(P);
  d.dsc[1] = al.get<double>(P);
  d.idx[0] = al.get<int32_t>(P);
  d.idx[1] = al.get<int32_t>(P);
  d.ord[0] = al.get<int32_t>(P);
  d.ord[1] = al.get<int32_t>(P);
  d.perm = al.get<int32_t>(P);
  d.Hp = al.get<double>(P * ENT_SEGS * 2);
  d.H = al.get<double>(P);
  d.eH = al.get<double>(P);
  d.eT = al.get<double>(P);
  d.Meps = al.get<double>(pp);
  d.Terr = al.get<double>(pp);
  d.eHp = al.get<double>(P);
  d.Mepsp = al.get<double>(pp);
  d.eTp = al.get<double>(P);
  d.Terrp = al.get<double>(pp);
  d.M = al.get<double>(pp);
  d.S = al.get<double>(P);
  d.alive = al.get<uint8_t>(P);
  d.alive_list = al.get<int32_t>(P);
  d.complete = al.get<uint8_t>(P);
  d.pend = al.get<uint8_t>(pp);
  d.P = al.get<double>((size_t)d.nchunk * pp * 4);
  d.ctl = ctl;
  d.order = al.get<int32_t>(P);
  d.Tall = al.get<double>(pp);
  d.Tstate = al.get<uint8_t>(pp);
  d.Hall = al.get<double>(pp);
  d.rec = o.record_M_iters;
  d.Mrec = d.rec > 0 ? al.get<double>((size_t)d.rec * pp) : nullptr;
  d.stats = al.get<double>(2 * P);
  d.gram_slices_max = GRAM_SLICES_MAX;
  d.Gp = al.get<double>((size_t)gram_partial_rows(p, n, GRAM_SLICES_MAX) * (size_t)p);
  d.forced_len = o.forced_len;
  int32_t* forced_dev = al.get<int32_t>(std::max<size_t>(1, (size_t)o.forced_len));
  d.forced = forced_dev;
  d.pair_slots = al.get<unsigned long long>(2 * PAIR_SLOTS);
  if (o.estimate_B) {
    d.C0 = al.get<double>(pp);
    d.Lch = al.get<double>(pp);
    d.Bout = al.get<double>(pp);
  }
  d.band_k0 = pl.band_blocks;
  d.messaging = o.messaging ? 1 : 0;
  d.band_adapt = o.band_blocks > 0 ? 0 : 1;
  return d;
}

// The forced prefix of the order (host memory of the caller) to the device;
// every other initial value is set by launch_init_sets.
void upload_forced(const Dev& d, const lingam_opts& o, hipStream_t s) {
  if (o.forced_len > 0)
    HIPCHK(hipMemcpyAsync(const_cast<int32_t*>(d.forced), o.forced_order, sizeof(int32_t) * o.forced_len,
                          hipMemcpyHostToDevice, s));
}

// Launch sequence of a batch (a single search is a batch of one).
struct Fit {
  PairTimer* timer = nullptr;
  Batch b;
  Plan pl;
  lingam_opts o;
  hipStream_t s;
  bool threshold;
  double gamma0, gmult;
  int rec = 0;
  std::vector<int64_t> ps;   // p of every data set
  std::vector<int> limits;   // iterations of every data set

  int slots = 0;             // band slots queued per iteration (0 = the most an iteration can use)
  int refresh_every = 1;     // Gram refresh period (0 = the rank-1 recursion only)

  void pair(int t, const BandArgs& a, bool dense, int ntb_hint) {
    if (o.pair_strategy != LINGAM_PAIR_DEFAULT) {
      HIPCHK(launch_pair_baseline(b, t, o.pair_strategy, a.chunk, s));
      return;
    }
    if (timer && timer->on) {
      hipEvent_t e0 = timer->next(), e1 = timer->next();
      HIPCHK(launch_pair_band(b, t, a, dense ? 1 : 0, ntb_hint, s, e0, e1));
      ++timer->launches;
    } else {
      HIPCHK(launch_pair_band(b, t, a, dense ? 1 : 0, ntb_hint, s));
    }
  }

  // one band slot: pair kernel then scores and decision
  void slot(int t, bool first) {
    const int r = b.p_max - t;
    const int nb = (r + TB - 1) / TB;
    const int hint = first ? (threshold ? std::min(pl.band_blocks, nb) : nb) : nb;
    BandArgs a{pl.chunk, 1, 1, BAND_TARGET_DEFAULT};
    pair_band_shape(b, a.rows_per_group, a.groups);
    if (b.count == 1 && b.mixed) a.band_target = band_target_single_mixed(b.p_max);
    if (o.band_target > 0.0) a.band_target = o.band_target;
    pair(t, a, first, hint);
    HIPCHK(launch_score(b, t, a, gmult, first ? 1 : 0, hint, s));
  }

  void queue_rounds(int t) {
    const int r = b.p_max - t;
    int n = threshold ? max_slots(r, pl.band_blocks) : 1;
    if (threshold && slots > 0) n = std::min(n, slots);
    for (int k = 0; k < n; ++k) slot(t, k == 0);
  }

  // after a host sync: size the next window's band slots from the most
  // bands one iteration of the last window needed (one spare)
  void update_slots(int win_bands) {
    if (win_bands > 0) slots = std::max(2, win_bands + 1);
    HIPCHK(launch_window_reset(b, s));
  }

  void queue_tail(int t) {
    const bool refresh = refresh_every > 0 && ((t + 1) % refresh_every == 0);
    HIPCHK(launch_iter_end(b, t, refresh ? 1 : 0, s));
    if (t < rec) HIPCHK(launch_record_M(b, t, s));
  }

  // iteration t of every data set that has one (p - t >= 2 and t < its limit);
  // a data set with one variable left appends it
  void queue_iteration(int t) {
    bool any_last = false;
    for (size_t k = 0; k < ps.size(); ++k) any_last |= (ps[k] - t == 1 && t < limits[k]);
    if (any_last) HIPCHK(launch_last(b, t, s));
    if (b.p_max - t < 2) return;
    // the previous iteration's row update summed the entropy terms unless a
    // Gram refresh followed it
    const int fused = t > 0 && !(refresh_every > 0 && t % refresh_every == 0) ? 1 : 0;
    HIPCHK(launch_iter_start(b, t, threshold ? gamma0 : INFINITY, GAMMA_ADAPT, threshold ? 1 : 0, fused, s));
    queue_rounds(t);
    queue_tail(t);
  }

  // Threshold rounds of iteration tf of a data set (a batch of one) that
  // halted because the queued rounds did not finish it, then its tail.
  Ctl finish_halted(Ctl* ctl_dev, int tf, int p) {
    HIPCHK(launch_resume(b, s));
    Ctl c{};
    for (int extra = 0;; ++extra) {
      slot(tf, false);
      c = read_ctl(ctl_dev);
      if (c.status != ST_OK || c.done) break;
      if (extra > p - tf + 8) throw HipFail{hipErrorUnknown, "threshold rounds did not terminate", __LINE__};
    }
    if (c.status == ST_OK) queue_tail(tf);
    return c;
  }

  Ctl read_ctl(Ctl* ctl_dev) {
    Ctl c;
    HIPCHK(hipMemcpyAsync(&c, ctl_dev, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return c;
  }

  // Iterations [t0, limit) of a batch of one, resuming halted iterations in
  // place.  Returns the final control block.
  Ctl drive_one(Ctl* ctl_dev, int t0, int limit, int p) {
    int t = t0;
    Ctl c{};
    while (t < limit) {
      for (int q = 0; q < SYNC_EVERY && t < limit; ++q, ++t) queue_iteration(t);
      c = read_ctl(ctl_dev);
      if (c.status != ST_OK) return c;
      update_slots(c.win_bands);
      if (c.halt && c.halt_iter >= 0) {
        // iteration halt_iter needed more threshold rounds than were queued;
        // every launch queued after it returned at once, so its state is intact.
        const int tf = c.halt_iter;
        c = finish_halted(ctl_dev, tf, p);
        if (c.status != ST_OK) return c;
        t = tf + 1;
      }
    }
    return read_ctl(ctl_dev);
  }
};

// The results of one data set in two steps, so that a batch waits once for
// all of its sets: queue the device-to-host copies (after launch_sum_slots),
// then, after the stream is synchronised, fill in the rest.
struct ResultCopy {
  unsigned long long slots[2];
};

void queue_results(const Dev& d, lingam_result* out, ResultCopy* rc, hipStream_t s) {
  const size_t P = (size_t)d.p, pp = P * P;
  HIPCHK(hipMemcpyAsync(out->order, d.order, sizeof(int32_t) * P, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(rc->slots, d.pair_slots, sizeof(rc->slots), hipMemcpyDeviceToHost, s));
  if (out->T) HIPCHK(hipMemcpyAsync(out->T, d.Tall, sizeof(double) * pp, hipMemcpyDeviceToHost, s));
  if (out->T_state) HIPCHK(hipMemcpyAsync(out->T_state, d.Tstate, pp, hipMemcpyDeviceToHost, s));
  if (out->H) HIPCHK(hipMemcpyAsync(out->H, d.Hall, sizeof(double) * pp, hipMemcpyDeviceToHost, s));
  if (out->T_err_bound)
    HIPCHK(hipMemcpyAsync(out->T_err_bound, d.Terr, sizeof(double) * pp, hipMemcpyDeviceToHost, s));
  if (out->T_err_prob)
    HIPCHK(hipMemcpyAsync(out->T_err_prob, d.Terrp, sizeof(double) * pp, hipMemcpyDeviceToHost, s));
  if (out->M && d.rec > 0)
    HIPCHK(hipMemcpyAsync(out->M, d.Mrec, sizeof(double) * pp * d.rec, hipMemcpyDeviceToHost, s));
}

void finish_results(const Dev& d, const Ctl& c, int64_t n, const ResultCopy& rc, lingam_result* out) {
  const size_t P = (size_t)d.p;
  out->pairs_evaluated = rc.slots[0];
  out->pair_samples = rc.slots[0] * (uint64_t)n;
  out->pairs_computed = rc.slots[1];
  out->threshold_rounds = c.rounds_total;
  out->bands = c.bands_total;
  int it = 0;
  for (size_t k = 0; k < P; ++k) if (out->order[k] >= 0) ++it;
  out->iterations = it;
  if (c.status != ST_OK) {
    out->bad_i = c.bad_i;
    out->bad_j = c.bad_j;
    out->status = c.status == ST_NONFINITE ? LINGAM_E_NONFINITE
                : c.status == ST_DEGENERATE ? LINGAM_E_DEGENERATE : LINGAM_E_INVALID;
  }
}

void copy_results(const Batch& b, const Dev& d, const Ctl& c, int64_t n, lingam_result* out, hipStream_t s) {
  ResultCopy rc{};
  HIPCHK(launch_sum_slots(b, s));
  queue_results(d, out, &rc, s);
  HIPCHK(hipStreamSynchronize(s));
  finish_results(d, c, n, rc, out);
}

lingam_status status_from(const HipFail& e) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s failed: %s (line %d)", e.what, hipGetErrorString(e.err), e.line);
  g_last_error = buf;
  return e.err == hipErrorOutOfMemory ? LINGAM_E_NOMEM : LINGAM_E_DEVICE;
}

void set_error_text(lingam_status st, const lingam_result* out) {
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s (variables %d, %d)", lingam_status_string(st), out->bad_i, out->bad_j);
  g_last_error = buf;
}


// ---- device memory of a call ---------------------------------------------

size_t x_bytes(int64_t n, int64_t p, const lingam_opts& o) {
  return (size_t)p * (size_t)n * (o.x_dtype == 1 ? 4 : 8);
}

// Buffers of a single search (one data set), in carve order.
struct SingleLayout {
  Ctl* ctl = nullptr;
  Dev d;
  void* xb = nullptr;   // staging of a host X
  Dev* dd = nullptr;    // device copy of the descriptor
};

SingleLayout layout_single(Arena& ar, int64_t n, int64_t p, const Plan& pl, const lingam_opts& o) {
  SingleLayout L;
  L.ctl = ar.get<Ctl>(1);
  L.d = carve_set(ar, n, p, pl, o, o.precision != LINGAM_PREC_FP64, L.ctl);
  if (!o.x_on_device) L.xb = ar.get<uint8_t>(x_bytes(n, p, o));
  L.dd = ar.get<Dev>(1);
  return L;
}

// Buffers of a batch, in carve order.  A bootstrap base (identified by its
// X pointer) is staged once; every bootstrap set gets its index vector and
// its gathered rows.
struct BatchLayout {
  Ctl* ctls = nullptr;
  std::vector<Dev> devs;
  std::vector<void*> xb;            // per set: staging of a host X (or nullptr)
  std::vector<const double*> base;  // per bootstrap set: its base rows on the device
  std::vector<char> base_upload;    // per set: 1 if this set's base is uploaded here
  std::vector<int64_t*> idx;        // per bootstrap set: device sample indices
  Dev* dd = nullptr;
  int32_t* act = nullptr;           // the sets in order of the iteration they end at (work queue)
};

BatchLayout layout_batch(Arena& ar, int32_t count, const lingam_dataset* sets, const Plan& pl,
                         const lingam_opts& o) {
  BatchLayout L;
  const bool mixed = o.precision != LINGAM_PREC_FP64;
  L.ctls = ar.get<Ctl>((size_t)count);
  L.devs.resize((size_t)count);
  L.xb.assign((size_t)count, nullptr);
  L.base.assign((size_t)count, nullptr);
  L.base_upload.assign((size_t)count, 0);
  L.idx.assign((size_t)count, nullptr);
  std::vector<std::pair<const void*, const double*>> bases;
  for (int k = 0; k < count; ++k) {
    const lingam_dataset& ds = sets[k];
    const int64_t nk = ds.sample_idx ? ds.n_idx : ds.n, pk = ds.p;
    Dev d = carve_set(ar, nk, pk, pl, o, mixed, L.ctls ? L.ctls + k : nullptr);
    if (ds.sample_idx) {
      const double* base = nullptr;
      bool found = false;
      for (auto& bp : bases)
        if (bp.first == ds.X) { base = bp.second; found = true; }
      if (!found) {
        if (o.x_on_device) {
          base = (const double*)ds.X;
        } else {
          base = ar.get<double>((size_t)pk * (size_t)ds.n);
          L.base_upload[(size_t)k] = 1;
        }
        bases.push_back({ds.X, base});
      }
      L.base[(size_t)k] = base;
      L.idx[(size_t)k] = ar.get<int64_t>((size_t)ds.n_idx);
      d.X = ar.get<double>((size_t)pk * (size_t)nk);   // the gathered resample
      d.x_dtype = 0;
      d.layout = 0;
    } else if (!o.x_on_device) {
      L.xb[(size_t)k] = ar.get<uint8_t>(x_bytes(nk, pk, o));
      d.X = L.xb[(size_t)k];
    } else {
      d.X = ds.X;
    }
    L.devs[(size_t)k] = d;
  }
  L.dd = ar.get<Dev>((size_t)count);
  L.act = ar.get<int32_t>((size_t)count);
  return L;
}

// Where a call's device memory comes from: the caller's workspace
// (opts.workspace), else one hipMalloc of the size the sizing pass found.
// Checks the caller's workspace on the host, before any device work.
lingam_status acquire(uint64_t need, const lingam_opts& o, OwnedMem& own, Arena& ar) {
  if (o.workspace) {
    if ((reinterpret_cast<uintptr_t>(o.workspace) & 255u) != 0)
      return fail(LINGAM_E_INVALID, "opts.workspace must be 256-byte aligned");
    if (o.workspace_bytes < need) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "opts.workspace holds %llu bytes, the call needs %llu",
                    (unsigned long long)o.workspace_bytes, (unsigned long long)need);
      return fail(LINGAM_E_NOMEM, buf);
    }
    ar.base = static_cast<char*>(o.workspace);
    ar.cap = o.workspace_bytes;
    return LINGAM_OK;
  }
  hipError_t e = hipMalloc(&own.p, need);
  if (e != hipSuccess) {
    own.p = nullptr;
    char buf[160];
    std::snprintf(buf, sizeof buf, "hipMalloc of %llu bytes failed: %s", (unsigned long long)need,
                  hipGetErrorString(e));
    return fail(e == hipErrorOutOfMemory ? LINGAM_E_NOMEM : LINGAM_E_DEVICE, buf);
  }
  ar.base = static_cast<char*>(own.p);
  ar.cap = need;
  return LINGAM_OK;
}

// One causal-order search.  fixed == nullptr: the device memory is the
// caller's workspace or one hipMalloc; otherwise it is the block
// [fixed->base, fixed->base + fixed->cap) on the current device, and the call
// allocates nothing (no device memory, streams or events are created; the
// search runs on opts.stream, NULL = the null stream).
// given_order (optional, host): skip the search and estimate B along this
// order (lingam_estimate_B).
lingam_status fit_single(const void* X, int64_t n, int64_t p, const lingam_opts& o, lingam_result* out,
                         const FixedBlock* fixed, const int32_t* given_order = nullptr) {
  const auto wall0 = std::chrono::steady_clock::now();
  g_last_error.clear();
  lingam_status st = validate(X, n, p, o, out);
  if (st != LINGAM_OK) return st;
  if (fixed) {
    if (o.workspace) return fail(LINGAM_E_INVALID, "this entry point takes no opts.workspace");
    if (o.profile) return fail(LINGAM_E_UNSUPPORTED, "opts.profile needs timing events, which allocate");
  }
  reset_result(out, p, o.record_M_iters);

  const Plan pl = make_plan(n, o, true);
  Arena sizing;
  (void)layout_single(sizing, n, p, pl, o);
  const uint64_t need = sizing.off;
  if (fixed && need > fixed->cap) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "p=%lld n=%lld needs %llu bytes of device memory; %s holds at most %llu",
                  (long long)p, (long long)n, (unsigned long long)need, fixed->who,
                  (unsigned long long)fixed->cap);
    return fail(LINGAM_E_NOMEM, buf);
  }

  OwnedMem own;
  OwnedStream os;
  PairTimer timer;
  DeviceGuard dg;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  const bool events = fixed == nullptr;
  try {
    dg.set(o.device);
    Arena ar;
    if (fixed) {
      ar.base = fixed->base;
      ar.cap = fixed->cap;
    } else {
      st = acquire(need, o, own, ar);
      if (st != LINGAM_OK) return st;
    }
    SingleLayout L = layout_single(ar, n, p, pl, o);
    if (o.stream || fixed) {
      os.s = (hipStream_t)o.stream;
    } else {
      HIPCHK(hipStreamCreate(&os.s));
      os.owned = true;
    }
    Fit f;
    f.timer = &timer;
    timer.on = o.profile != 0;
    f.o = o;
    f.s = os.s;
    f.refresh_every = o.cov_refresh_every >= 0 ? o.cov_refresh_every
                      : (o.precision != LINGAM_PREC_FP64 ? REFRESH_MIXED : 1);
    const bool mixed = o.precision != LINGAM_PREC_FP64;
    f.threshold = o.use_threshold != 0;
    f.gamma0 = o.gamma0 > 0 ? o.gamma0 : 0.0;  // 0 = adaptive
    f.gmult = o.gamma_mult > 1.0 ? o.gamma_mult : 4.0;
    f.pl = pl;
    f.rec = o.record_M_iters;
    const int limit = (o.max_roots > 0 && o.max_roots < p) ? o.max_roots : (int)p;
    f.ps = {p};
    f.limits = {limit};

    Dev& d = L.d;
    d.limit = limit;
    if (!o.x_on_device) {
      HIPCHK(hipMemcpyAsync(L.xb, X, x_bytes(n, p, o), hipMemcpyHostToDevice, f.s));
      d.X = L.xb;
    } else {
      d.X = X;
    }
    // (L.d stays alive for the whole call, so the copy needs no wait)
    HIPCHK(hipMemcpyAsync(L.dd, &d, sizeof(Dev), hipMemcpyHostToDevice, f.s));
    upload_forced(d, o, f.s);

    f.b.dd = L.dd;
    f.b.count = 1;
    f.b.one = d;
    f.b.p_max = (int)p;
    f.b.n_max = n;
    f.b.nchunk_max = d.nchunk;
    f.b.gram_slices_max = GRAM_SLICES_MAX;
    f.b.mixed = mixed ? 1 : 0;
    f.b.store32 = o.precision == LINGAM_PREC_FP32_STORAGE ? 1 : 0;
    f.b.queue = o.batch_queue ? 1 : 0;
    HIPCHK(launch_init_sets(f.b, f.s));

    if (events) {
      HIPCHK(hipEventCreate(&ev0));
      HIPCHK(hipEventCreate(&ev1));
      HIPCHK(hipEventRecord(ev0, f.s));
    }
    // a1 + a2: normalise once, covariance once (Alg. 3)
    HIPCHK(launch_standardize(f.b, f.s));
    HIPCHK(launch_gram(f.b, 0, 0, f.s));
    if (o.estimate_B) HIPCHK(launch_corr_snapshot(d, f.s));
    Ctl c;
    if (given_order) {
      HIPCHK(hipMemcpyAsync(d.order, given_order, sizeof(int32_t) * p, hipMemcpyHostToDevice, f.s));
      c = f.read_ctl(L.ctl);
    } else {
      c = f.drive_one(L.ctl, 0, limit, (int)p);
    }
    // Alg. 1, last step: the causal strengths along the order
    if (o.estimate_B && c.status == ST_OK) {
      HIPCHK(launch_estimate_B(d, f.s));
      c = f.read_ctl(L.ctl);
      if (c.status == ST_OK)
        HIPCHK(hipMemcpyAsync(out->B, d.Bout, sizeof(double) * p * p, hipMemcpyDeviceToHost, f.s));
    }
    if (events) HIPCHK(hipEventRecord(ev1, f.s));
    copy_results(f.b, d, c, n, out, f.s);
    float ms = 0.f;
    if (events && hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) out->seconds_device = ms * 1e-3;
    if (timer.on) {
      out->seconds_pair_kernel = timer.total_seconds();
      out->pair_kernel_launches = timer.launches;
    }
    st = (lingam_status)out->status;
    if (st != LINGAM_OK) set_error_text(st, out);
  } catch (const HipFail& e) {
    st = status_from(e);
    out->status = st;
  } catch (const NoMem& e) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "workspace layout needs %llu bytes, %llu available",
                  (unsigned long long)e.need, (unsigned long long)e.have);
    st = fail(LINGAM_E_NOMEM, buf);
    out->status = st;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  out->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  return st;
}

// ---- hipGraph windows of batched searches ----------------------------------
// The launches of a window of SYNC_EVERY iterations of a batch depend only
// on the layout of the call's device memory (its base address and the data
// sets' shapes), the options and the window (first iteration, length, band
// slots per iteration).  With opts.graph the window is captured into a graph
// once and replayed by later calls whose memory has the same address and
// layout (a caller's workspace, or a repeated allocation at the same
// address); every graph is a chain of kernel nodes (the buffers are set by
// fill kernels outside the windows, never by memset nodes).
// The cache lives until the process ends and its graphs are not destroyed
// at exit (the HIP runtime may already be torn down by then); it is
// cleared whenever it reaches GRAPH_CACHE_MAX entries.
struct GraphCache {
  std::mutex mu;
  std::unordered_map<uint64_t, hipGraphExec_t> execs;
};
GraphCache g_graphs;
constexpr size_t GRAPH_CACHE_MAX = 4096;

uint64_t mix64(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h * 0xff51afd7ed558ccdull;
}

uint64_t batch_layout_key(const char* base, uint64_t bytes, int32_t count, const lingam_dataset* sets,
                          const lingam_opts& o, int refresh_every, const Plan& pl) {
  // an instantiated graph belongs to the device it was captured on
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  uint64_t h = mix64((uint64_t)(uint32_t)dev, reinterpret_cast<uintptr_t>(base));
  h = mix64(h, bytes);
  h = mix64(h, (uint64_t)count);
  for (int k = 0; k < count; ++k) {
    h = mix64(h, (uint64_t)sets[k].p);
    h = mix64(h, (uint64_t)(sets[k].sample_idx ? sets[k].n_idx : sets[k].n));
    int first = k;   // the first set with the same base (bootstrap bases are staged once)
    if (sets[k].sample_idx)
      for (int j = 0; j < k; ++j)
        if (sets[j].sample_idx && sets[j].X == sets[k].X) { first = j; break; }
    h = mix64(h, (uint64_t)first * 2 + (sets[k].sample_idx ? 1 : 0));
  }
  const uint64_t fields[] = {(uint64_t)o.precision, (uint64_t)o.use_threshold, (uint64_t)o.max_roots,
                             (uint64_t)o.batch_queue, (uint64_t)refresh_every, (uint64_t)pl.chunk,
                             (uint64_t)pl.band_blocks, (uint64_t)o.band_blocks, (uint64_t)o.first_band_blocks,
                             (uint64_t)o.x_dtype, (uint64_t)o.messaging, (uint64_t)o.pair_strategy,
                             (uint64_t)o.layout, (uint64_t)o.x_on_device};
  for (uint64_t v : fields) h = mix64(h, v);
  uint64_t g0, gm, bt;
  std::memcpy(&g0, &o.gamma0, 8);
  std::memcpy(&gm, &o.gamma_mult, 8);
  std::memcpy(&bt, &o.band_target, 8);
  return mix64(mix64(mix64(h, g0), gm), bt);
}

// Queue iterations [t, t + nwin) of f on its stream: replayed from the cache
// or captured and kept when `graph` is set, launched one by one otherwise.
void queue_window(Fit& f, int t, int nwin, bool graph, uint64_t layout_key) {
  if (!graph) {
    for (int q = 0; q < nwin; ++q) f.queue_iteration(t + q);
    return;
  }
  const uint64_t key = mix64(mix64(mix64(layout_key, (uint64_t)t), (uint64_t)nwin), (uint64_t)f.slots);
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_graphs.mu);
    auto it = g_graphs.execs.find(key);
    if (it != g_graphs.execs.end()) exec = it->second;
  }
  if (!exec) {
    HIPCHK(hipStreamBeginCapture(f.s, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      for (int q = 0; q < nwin; ++q) f.queue_iteration(t + q);
    } catch (...) {
      (void)hipStreamEndCapture(f.s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(f.s, &g));
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw HipFail{e, "hipGraphInstantiate", __LINE__};
    std::lock_guard<std::mutex> lk(g_graphs.mu);
    if (g_graphs.execs.size() >= GRAPH_CACHE_MAX) {
      for (auto& kv : g_graphs.execs) (void)hipGraphExecDestroy(kv.second);
      g_graphs.execs.clear();
    }
    g_graphs.execs[key] = exec;
  }
  HIPCHK(hipGraphLaunch(exec, f.s));
}

lingam_status validate_batch(int32_t count, const lingam_dataset* sets, const lingam_opts& o,
                             const lingam_result* outs) {
  if (count < 1 || !sets) return fail(LINGAM_E_INVALID, "empty batch or NULL arrays");
  if (count > 65535) return fail(LINGAM_E_INVALID, "at most 65535 data sets per batch");
  lingam_status st = validate_opts(o);
  if (st != LINGAM_OK) return st;
  if (o.forced_len > 0 || o.record_M_iters > 0 || o.estimate_B)
    return fail(LINGAM_E_UNSUPPORTED, "forced_order, record_M_iters and estimate_B are not available in batches");
  if (o.pair_strategy != LINGAM_PAIR_DEFAULT)
    return fail(LINGAM_E_UNSUPPORTED, "the baseline pair strategies are not available in batches");
  for (int k = 0; k < count; ++k) {
    const lingam_dataset& ds = sets[k];
    if (!ds.X) return fail(LINGAM_E_INVALID, "data set with X == NULL");
    if (outs && !outs[k].order) return fail(LINGAM_E_INVALID, "result->order is NULL");
    const int64_t nk = ds.sample_idx ? ds.n_idx : ds.n;
    st = validate_shape(nk, ds.p);
    if (st != LINGAM_OK) return st;
    if (ds.sample_idx) {
      if (ds.n < 1) return fail(LINGAM_E_INVALID, "bootstrap base with n < 1");
      if (o.x_dtype != 0 || o.layout != LINGAM_LAYOUT_VAR_MAJOR)
        return fail(LINGAM_E_UNSUPPORTED, "bootstrap data sets need a binary64 p x n base");
      for (int64_t i = 0; i < ds.n_idx; ++i)
        if (ds.sample_idx[i] < 0 || ds.sample_idx[i] >= ds.n)
          return fail(LINGAM_E_INVALID, "bootstrap sample index out of range");
    }
  }
  return LINGAM_OK;
}

Plan batch_plan(int32_t count, const lingam_dataset* sets, const lingam_opts& o) {
  int64_t n_max = 0;
  for (int k = 0; k < count; ++k) n_max = std::max(n_max, sets[k].sample_idx ? sets[k].n_idx : sets[k].n);
  return make_plan(n_max, o, false);  // the chunk length is the same for every data set
}

}  // namespace

namespace lingam {
lingam_status fit_order_in_block(const void* X, int64_t n, int64_t p, const lingam_opts* opts,
                                 lingam_result* out, const FixedBlock& block) {
  lingam_opts o;
  if (opts) o = *opts; else lingam_opts_default(&o);
  return fit_single(X, n, p, o, out, &block);
}
void set_last_error(const char* msg) { g_last_error = msg; }
}  // namespace lingam

extern "C" {

void lingam_opts_default(lingam_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(lingam_opts);
  o->precision = LINGAM_PREC_FP64;
  o->layout = LINGAM_LAYOUT_VAR_MAJOR;
  o->x_dtype = 0;
  o->x_on_device = 0;
  o->device = -1;
  o->use_threshold = 1;
  o->gamma0 = 0.0;
  o->gamma_mult = 4.0;
  o->cov_refresh_every = -1;
  o->max_roots = 0;
  o->forced_order = nullptr;
  o->forced_len = 0;
  o->record_M_iters = 0;
  o->band_blocks = 0;
  o->chunk_samples = 0;
  o->stream = nullptr;
  o->profile = 0;
  o->batch_queue = 1;
  o->messaging = 1;
}

const char* lingam_status_string(lingam_status s) {
  switch (s) {
    case LINGAM_OK: return "ok";
    case LINGAM_E_INVALID: return "invalid argument";
    case LINGAM_E_NONFINITE: return "non-finite value in X";
    case LINGAM_E_DEGENERATE: return "degenerate input (zero variance or collinear pair)";
    case LINGAM_E_NOMEM: return "out of device memory";
    case LINGAM_E_DEVICE: return "HIP device error";
    case LINGAM_E_UNSUPPORTED: return "unsupported option combination";
  }
  return "unknown status";
}

const char* lingam_last_error(void) { return g_last_error.c_str(); }

uint64_t lingam_workspace_size(int64_t n, int64_t p, const lingam_opts* o) {
  lingam_opts def;
  lingam_opts_default(&def);
  const lingam_opts& op = o ? *o : def;
  if (n < 2 || p < 1) return 0;
  Arena sizing;
  (void)layout_single(sizing, n, p, make_plan(n, op, true), op);
  return sizing.off;
}

uint64_t lingam_workspace_size_batch(int32_t count, const lingam_dataset* sets, const lingam_opts* o) {
  lingam_opts def;
  lingam_opts_default(&def);
  const lingam_opts& op = o ? *o : def;
  if (validate_batch(count, sets, op, nullptr) != LINGAM_OK) return 0;
  Arena sizing;
  (void)layout_batch(sizing, count, sets, batch_plan(count, sets, op), op);
  return sizing.off;
}

lingam_status lingam_fit_order(const void* X, int64_t n, int64_t p, const lingam_opts* opts,
                               lingam_result* out) {
  lingam_opts o;
  if (opts) o = *opts; else lingam_opts_default(&o);
  return fit_single(X, n, p, o, out, nullptr);
}

lingam_status lingam_estimate_B(const void* X, int64_t n, int64_t p, const int32_t* order,
                                const lingam_opts* opts, double* B) {
  g_last_error.clear();
  lingam_opts o;
  if (opts) o = *opts; else lingam_opts_default(&o);
  if (!order || !B) return fail(LINGAM_E_INVALID, "order or B is NULL");
  if (p < 1 || p > B_MAX_P) return fail(LINGAM_E_INVALID, "estimate_B supports 1 <= p <= 8000");
  std::vector<char> seen((size_t)p, 0);
  for (int64_t k = 0; k < p; ++k) {
    const int32_t v = order[k];
    if (v < 0 || v >= p || seen[(size_t)v]) return fail(LINGAM_E_INVALID, "order is not a permutation");
    seen[(size_t)v] = 1;
  }
  o.estimate_B = 1;
  o.max_roots = 0;
  o.forced_len = 0;
  o.forced_order = nullptr;
  o.record_M_iters = 0;
  std::vector<int32_t> ord((size_t)p);
  lingam_result res;
  std::memset(&res, 0, sizeof(res));
  res.order = ord.data();
  res.B = B;
  return fit_single(X, n, p, o, &res, nullptr, order);
}

lingam_status lingam_check_terms(int32_t device, lingam_term_check* out) {
  g_last_error.clear();
  if (!out) return fail(LINGAM_E_INVALID, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  OwnedMem own;
  OwnedStream os;
  DeviceGuard dg;
  try {
    dg.set(device);
    HIPCHK(hipMalloc(&own.p, sizeof(TermSweep)));
    HIPCHK(hipStreamCreate(&os.s));
    os.owned = true;
    HIPCHK(launch_fill_u8(static_cast<uint8_t*>(own.p), sizeof(TermSweep), 0, os.s));
    HIPCHK(launch_term_sweep(static_cast<TermSweep*>(own.p), os.s));
    TermSweep r;
    HIPCHK(hipMemcpyAsync(&r, own.p, sizeof(TermSweep), hipMemcpyDeviceToHost, os.s));
    HIPCHK(hipStreamSynchronize(os.s));
    double mx[2];
    std::memcpy(mx, r.max_bits, sizeof(mx));
    const uint64_t exp_count = 0x42FC0000ull + 1, log_count = 0x40000000ull - 0x3F800000ull + 1;
    out->exp2_max_rel = mx[0];
    out->exp2_mean_rel = r.sum[0] / (double)exp_count;
    out->log2_max_abs = mx[1];
    out->log2_mean_abs = r.sum[1] / (double)log_count;
    out->exp2_count = exp_count;
    out->log2_count = log_count;
    // binades of |x|: exponent fields 0 (zero and subnormals) .. 132 hold 2^23
    // arguments each, field 133 ([64, 126]) the rest
    for (int e = 0; e <= 133; ++e) {
      const double cnt = e < 133 ? 8388608.0 : (double)(0x42FC0000ull - 0x42800000ull + 1);
      out->exp2_max_binade_mean = std::max(out->exp2_max_binade_mean, std::fabs(r.binade_sum[0][e] / cnt));
    }
  } catch (const HipFail& e) {
    return status_from(e);
  }
  return LINGAM_OK;
}

lingam_status lingam_fit_order_batch(int32_t count, const lingam_dataset* sets, const lingam_opts* opts,
                                     lingam_result* outs) {
  const auto wall0 = std::chrono::steady_clock::now();
  g_last_error.clear();
  lingam_opts o;
  if (opts) o = *opts; else lingam_opts_default(&o);
  if (!outs) return fail(LINGAM_E_INVALID, "empty batch or NULL arrays");
  lingam_status st = validate_batch(count, sets, o, outs);
  if (st != LINGAM_OK) return st;
  for (int k = 0; k < count; ++k) reset_result(&outs[k], sets[k].p, 0);

  const Plan pl = batch_plan(count, sets, o);
  Arena sizing;
  (void)layout_batch(sizing, count, sets, pl, o);
  const uint64_t need = sizing.off;

  OwnedMem own;
  OwnedStream os;
  PairTimer timer;
  DeviceGuard dg;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  try {
    dg.set(o.device);
    Arena ar;
    st = acquire(need, o, own, ar);
    if (st != LINGAM_OK) return st;
    BatchLayout L = layout_batch(ar, count, sets, pl, o);
    if (o.stream) {
      os.s = (hipStream_t)o.stream;
    } else {
      HIPCHK(hipStreamCreate(&os.s));
      os.owned = true;
    }
    Fit f;
    f.timer = &timer;
    timer.on = o.profile != 0;
    f.o = o;
    f.s = os.s;
    f.refresh_every = o.cov_refresh_every >= 0 ? o.cov_refresh_every
                      : (o.precision != LINGAM_PREC_FP64 ? REFRESH_MIXED : 1);
    const bool mixed = o.precision != LINGAM_PREC_FP64;
    f.threshold = o.use_threshold != 0;
    f.gamma0 = o.gamma0 > 0 ? o.gamma0 : 0.0;
    f.gmult = o.gamma_mult > 1.0 ? o.gamma_mult : 4.0;
    f.pl = pl;
    int64_t p_max = 0, n_max = 0;
    for (int k = 0; k < count; ++k) {
      p_max = std::max(p_max, sets[k].p);
      n_max = std::max(n_max, sets[k].sample_idx ? sets[k].n_idx : sets[k].n);
    }
    f.ps.resize((size_t)count);
    f.limits.resize((size_t)count);
    int nchunk_max = 1;
    for (int k = 0; k < count; ++k) {
      const lingam_dataset& ds = sets[k];
      const int64_t nk = ds.sample_idx ? ds.n_idx : ds.n, pk = ds.p;
      const int limit = (o.max_roots > 0 && o.max_roots < pk) ? o.max_roots : (int)pk;
      Dev& d = L.devs[(size_t)k];
      d.limit = limit;
      if (ds.sample_idx) {
        if (L.base_upload[(size_t)k])
          HIPCHK(hipMemcpyAsync(const_cast<double*>(L.base[(size_t)k]), ds.X, sizeof(double) * pk * ds.n,
                                hipMemcpyHostToDevice, f.s));
        HIPCHK(hipMemcpyAsync(L.idx[(size_t)k], ds.sample_idx, sizeof(int64_t) * ds.n_idx,
                              hipMemcpyHostToDevice, f.s));
        HIPCHK(launch_gather(L.base[(size_t)k], ds.n, pk, L.idx[(size_t)k], nk,
                             const_cast<double*>(static_cast<const double*>(d.X)), f.s));
      } else if (L.xb[(size_t)k]) {
        HIPCHK(hipMemcpyAsync(L.xb[(size_t)k], ds.X, x_bytes(nk, pk, o), hipMemcpyHostToDevice, f.s));
      }
      f.ps[(size_t)k] = pk;
      f.limits[(size_t)k] = limit;
      nchunk_max = std::max(nchunk_max, d.nchunk);
    }
    Ctl* ctls = L.ctls;
    Dev* dd = L.dd;
    std::vector<Dev>& devs = L.devs;
    HIPCHK(hipMemcpyAsync(dd, devs.data(), sizeof(Dev) * count, hipMemcpyHostToDevice, f.s));

    // the work queue's list of sets, latest-ending first: the sets with an
    // iteration at t are a prefix of it
    std::vector<int32_t> act_order((size_t)count);
    std::vector<int> act_until((size_t)count);
    for (int k = 0; k < count; ++k) act_order[(size_t)k] = k;
    auto until = [&](int k) { return std::min(f.limits[(size_t)k], (int)f.ps[(size_t)k] - 1); };
    std::stable_sort(act_order.begin(), act_order.end(), [&](int x, int y) { return until(x) > until(y); });
    for (int k = 0; k < count; ++k) act_until[(size_t)k] = until(act_order[(size_t)k]);
    HIPCHK(hipMemcpyAsync(L.act, act_order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, f.s));
    HIPCHK(hipStreamSynchronize(f.s));
    f.b.act = L.act;
    f.b.act_until = act_until.data();
    f.b.dd = dd;
    f.b.count = count;
    f.b.p_max = (int)p_max;
    f.b.n_max = n_max;
    f.b.nchunk_max = nchunk_max;
    f.b.gram_slices_max = GRAM_SLICES_MAX;
    f.b.mixed = mixed ? 1 : 0;
    f.b.store32 = o.precision == LINGAM_PREC_FP32_STORAGE ? 1 : 0;
    f.b.queue = o.batch_queue ? 1 : 0;
    int limit_max = 0;
    for (int l : f.limits) limit_max = std::max(limit_max, l);
    HIPCHK(launch_init_sets(f.b, f.s));

    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, f.s));
    HIPCHK(launch_standardize(f.b, f.s));
    HIPCHK(launch_gram(f.b, 0, 0, f.s));
    // every data set steps through its iterations together; one that halts
    // (not enough threshold rounds queued, or an error) sits out from then on
    std::vector<Ctl> cs((size_t)count);
    const bool graph = o.graph != 0 && !timer.on;
    const uint64_t lkey = graph ? batch_layout_key(ar.base, need, count, sets, o, f.refresh_every, pl) : 0;
    for (int t = 0; t < limit_max;) {
      const int nwin = std::min(SYNC_EVERY, limit_max - t);
      queue_window(f, t, nwin, graph, lkey);
      t += nwin;
      HIPCHK(hipMemcpyAsync(cs.data(), ctls, sizeof(Ctl) * count, hipMemcpyDeviceToHost, f.s));
      HIPCHK(hipStreamSynchronize(f.s));
      int wb = 0;
      for (const Ctl& c : cs) wb = std::max(wb, (int)c.win_bands);
      f.update_slots(wb);
    }
    // stragglers: finish each one alone, from the iteration that halted
    for (int k = 0; k < count; ++k) {
      if (cs[(size_t)k].status != ST_OK || !(cs[(size_t)k].halt && cs[(size_t)k].halt_iter >= 0)) continue;
      Fit g = f;
      g.b.dd = dd + k;
      g.b.count = 1;
      g.b.one = devs[(size_t)k];
      g.b.p_max = (int)sets[k].p;
      g.b.n_max = devs[(size_t)k].n;
      g.b.nchunk_max = devs[(size_t)k].nchunk;
      g.ps = {sets[k].p};
      g.limits = {f.limits[(size_t)k]};
      const int tf = cs[(size_t)k].halt_iter;
      Ctl c = g.finish_halted(ctls + k, tf, (int)sets[k].p);
      if (c.status == ST_OK) g.drive_one(ctls + k, tf + 1, f.limits[(size_t)k], (int)sets[k].p);
    }
    HIPCHK(hipEventRecord(ev1, f.s));
    // every set's results in one wait
    HIPCHK(launch_sum_slots(f.b, f.s));
    HIPCHK(hipMemcpyAsync(cs.data(), ctls, sizeof(Ctl) * count, hipMemcpyDeviceToHost, f.s));
    std::vector<ResultCopy> rcs((size_t)count);
    for (int k = 0; k < count; ++k) queue_results(devs[(size_t)k], &outs[k], &rcs[(size_t)k], f.s);
    HIPCHK(hipStreamSynchronize(f.s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    st = LINGAM_OK;
    for (int k = 0; k < count; ++k) {
      finish_results(devs[(size_t)k], cs[(size_t)k], devs[(size_t)k].n, rcs[(size_t)k], &outs[k]);
      outs[k].seconds_device = ms * 1e-3;
      if (timer.on) {
        outs[k].seconds_pair_kernel = timer.total_seconds();
        outs[k].pair_kernel_launches = timer.launches;
      }
      if (outs[k].status != LINGAM_OK && st == LINGAM_OK) {
        st = (lingam_status)outs[k].status;
        set_error_text(st, &outs[k]);
      }
    }
  } catch (const HipFail& e) {
    st = status_from(e);
    for (int k = 0; k < count; ++k) outs[k].status = st;
  } catch (const NoMem& e) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "workspace layout needs %llu bytes, %llu available",
                  (unsigned long long)e.need, (unsigned long long)e.have);
    st = fail(LINGAM_E_NOMEM, buf);
    for (int k = 0; k < count; ++k) outs[k].status = st;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  for (int k = 0; k < count; ++k) outs[k].seconds_total = wall;
  return st;
}

}  // extern "C"
