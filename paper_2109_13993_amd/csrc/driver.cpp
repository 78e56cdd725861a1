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

// Device allocations of one call, released on every exit path.
struct Allocs {
  std::vector<void*> ptrs;
  ~Allocs() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <class T>
  T* get(size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) throw HipFail{e, "hipMalloc", __LINE__};
    ptrs.push_back(q);
    return static_cast<T*>(q);
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
  if (o.precision == LINGAM_PREC_MIXED) chunk = std::min(chunk, CHUNK_MAX_MIXED);
  pl.chunk = chunk;
  pl.nchunk = (int)((n + chunk - 1) / chunk);
  pl.band_blocks = o.band_blocks > 0 ? o.band_blocks
                 : (single && o.precision == LINGAM_PREC_MIXED ? BAND_BLOCKS_SINGLE_MIXED : BAND_BLOCKS_DEFAULT);
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
  if (o.precision != LINGAM_PREC_FP64 && o.precision != LINGAM_PREC_MIXED)
    return fail(LINGAM_E_INVALID, "unknown precision");
  if (o.layout != LINGAM_LAYOUT_VAR_MAJOR && o.layout != LINGAM_LAYOUT_SAMPLE_MAJOR)
    return fail(LINGAM_E_INVALID, "unknown layout");
  if (o.x_dtype != 0 && o.x_dtype != 1) return fail(LINGAM_E_INVALID, "x_dtype must be 0 or 1");
  if (o.max_roots < 0) return fail(LINGAM_E_INVALID, "max_roots < 0");
  if (o.chunk_samples < 0 || o.chunk_samples % SUB != 0)
    return fail(LINGAM_E_INVALID, "chunk_samples must be a multiple of 256");
  if (o.band_blocks < 0) return fail(LINGAM_E_INVALID, "band_blocks < 0");
  if (o.record_M_iters < 0) return fail(LINGAM_E_INVALID, "record_M_iters < 0");
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

Dev alloc_set(Allocs& al, int64_t n, int64_t p, const Plan& pl, const lingam_opts& o, bool mixed, Ctl* ctl) {
  Dev d;
  d.p = (int)p;
  d.n = n;
  d.ldz = round_up(n, SUB);
  d.nchunk = (int)((n + pl.chunk - 1) / pl.chunk);
  d.mixed = mixed ? 1 : 0;
  d.x_dtype = o.x_dtype;
  d.layout = o.layout;
  const size_t P = (size_t)p, pp = P * P;
  d.Z[0] = al.get<double>(P * d.ldz);
  d.Z[1] = al.get<double>(P * d.ldz);
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
  d.Gp = al.get<double>((size_t)GRAM_SLICES_MAX * pp);
  d.forced_len = o.forced_len;
  int32_t* forced_dev = al.get<int32_t>(std::max<size_t>(1, (size_t)o.forced_len));
  d.forced = forced_dev;
  d.pair_slots = al.get<unsigned long long>(2 * PAIR_SLOTS);
  d.band_k0 = pl.band_blocks;
  d.band_adapt = o.band_blocks > 0 ? 0 : 1;
  return d;
}

// Initial contents of one data set's buffers (queued on s; fills by kernel,
// no memset nodes).
void init_set(const Dev& d, const lingam_opts& o, int limit, hipStream_t s, std::vector<int32_t>& iota) {
  const size_t P = (size_t)d.p, pp = P * P;
  if (o.forced_len > 0)
    HIPCHK(hipMemcpyAsync(const_cast<int32_t*>(d.forced), o.forced_order, sizeof(int32_t) * o.forced_len,
                          hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d.idx[0], iota.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d.ord[0], iota.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, s));
  HIPCHK(launch_fill(d.Z[1], (int64_t)(P * d.ldz), 0.0, s));
  HIPCHK(launch_fill(d.M, (int64_t)pp, NAN, s));
  HIPCHK(launch_fill_u8(d.pend, (int64_t)pp, 0, s));
  HIPCHK(launch_fill(d.Tall, (int64_t)pp, NAN, s));
  HIPCHK(launch_fill_u8(d.Tstate, (int64_t)pp, 0, s));
  HIPCHK(launch_fill(d.Hall, (int64_t)pp, NAN, s));
  HIPCHK(launch_fill(d.Terr, (int64_t)pp, NAN, s));
  if (d.Mrec) HIPCHK(launch_fill(d.Mrec, (int64_t)d.rec * (int64_t)pp, NAN, s));
  HIPCHK(launch_fill_u8(reinterpret_cast<uint8_t*>(d.order), (int64_t)(4 * P), 0xff, s));
  HIPCHK(launch_fill_u8(reinterpret_cast<uint8_t*>(d.pair_slots), (int64_t)(2 * PAIR_SLOTS * 8), 0, s));
  (void)limit;
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
    if (b.count == 1 && b.mixed) a.band_target = BAND_TARGET_SINGLE_MIXED;
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

void copy_results(const Dev& d, const Ctl& c, int64_t n, lingam_result* out, hipStream_t s) {
  const size_t P = (size_t)d.p, pp = P * P;
  std::vector<int32_t> order(P);
  std::vector<unsigned long long> slots(2 * PAIR_SLOTS);
  HIPCHK(hipMemcpyAsync(order.data(), d.order, sizeof(int32_t) * P, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(slots.data(), d.pair_slots, sizeof(unsigned long long) * 2 * PAIR_SLOTS,
                        hipMemcpyDeviceToHost, s));
  if (out->T) HIPCHK(hipMemcpyAsync(out->T, d.Tall, sizeof(double) * pp, hipMemcpyDeviceToHost, s));
  if (out->T_state) HIPCHK(hipMemcpyAsync(out->T_state, d.Tstate, pp, hipMemcpyDeviceToHost, s));
  if (out->H) HIPCHK(hipMemcpyAsync(out->H, d.Hall, sizeof(double) * pp, hipMemcpyDeviceToHost, s));
  if (out->T_err_bound)
    HIPCHK(hipMemcpyAsync(out->T_err_bound, d.Terr, sizeof(double) * pp, hipMemcpyDeviceToHost, s));
  if (out->M && d.rec > 0)
    HIPCHK(hipMemcpyAsync(out->M, d.Mrec, sizeof(double) * pp * d.rec, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::memcpy(out->order, order.data(), sizeof(int32_t) * P);
  uint64_t ev = 0, comp = 0;
  for (int k = 0; k < PAIR_SLOTS; ++k) {
    ev += slots[(size_t)k];
    comp += slots[(size_t)(PAIR_SLOTS + k)];
  }
  out->pairs_evaluated = ev;
  out->pair_samples = ev * (uint64_t)n;
  out->pairs_computed = comp;
  out->threshold_rounds = c.rounds_total;
  out->bands = c.bands_total;
  int it = 0;
  for (size_t k = 0; k < P; ++k) if (order[k] >= 0) ++it;
  out->iterations = it;
  if (c.status != ST_OK) {
    out->bad_i = c.bad_i;
    out->bad_j = c.bad_j;
    out->status = c.status == ST_NONFINITE ? LINGAM_E_NONFINITE
                : c.status == ST_DEGENERATE ? LINGAM_E_DEGENERATE : LINGAM_E_INVALID;
  }
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

}  // namespace

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
  const Plan pl = make_plan(n, op, true);
  const uint64_t ldz = (uint64_t)round_up(n, SUB);
  const uint64_t P = (uint64_t)p, pp = P * P;
  uint64_t b = 0;
  b += 2 * P * ldz * 8;                 // Z
  b += 2 * pp * 8 + 5 * P * 4;          // Sigma, idx, ord, perm
  b += P * ENT_SEGS * 16;               // entropy sums of the updated rows
  b += pp * 8 + pp;                     // M, pend
  b += (uint64_t)pl.nchunk * pp * 32;   // partials
  b += 4 * P * 8 + 2 * P;               // H, S, stats, alive/complete
  b += 16 * pp * 8 + 2 * P * 8;         // split-Gram partials, row scales
  b += pp * (8 + 1 + 8) + P * 4;        // T, T_state, H record, order
  b += 2 * pp * 8 + 2 * P * 8;          // rounding bounds: per test, per score record, eH, eT
  b += (uint64_t)op.record_M_iters * pp * 8;
  if (!op.x_on_device) b += P * (uint64_t)n * (op.x_dtype == 1 ? 4 : 8);
  b += sizeof(Ctl) + sizeof(Dev) + 2 * PAIR_SLOTS * 8;
  return b;
}

lingam_status lingam_fit_order(const void* X, int64_t n, int64_t p, const lingam_opts* opts,
                               lingam_result* out) {
  const auto wall0 = std::chrono::steady_clock::now();
  g_last_error.clear();
  lingam_opts o;
  if (opts) o = *opts; else lingam_opts_default(&o);
  lingam_status st = validate(X, n, p, o, out);
  if (st != LINGAM_OK) return st;
  reset_result(out, p, o.record_M_iters);

  Allocs al;
  OwnedStream os;
  PairTimer timer;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  try {
    if (o.device >= 0) HIPCHK(hipSetDevice(o.device));
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
                      : (o.precision == LINGAM_PREC_MIXED ? REFRESH_MIXED : 1);
    const bool mixed = o.precision == LINGAM_PREC_MIXED;
    f.threshold = o.use_threshold != 0;
    f.gamma0 = o.gamma0 > 0 ? o.gamma0 : 0.0;  // 0 = adaptive
    f.gmult = o.gamma_mult > 1.0 ? o.gamma_mult : 4.0;
    f.pl = make_plan(n, o, true);
    f.rec = o.record_M_iters;
    const int limit = (o.max_roots > 0 && o.max_roots < p) ? o.max_roots : (int)p;
    f.ps = {p};
    f.limits = {limit};

    Ctl* ctl = al.get<Ctl>(1);
    Dev d = alloc_set(al, n, p, f.pl, o, mixed, ctl);
    d.limit = limit;
    if (!o.x_on_device) {
      const size_t bytes = (size_t)p * (size_t)n * (o.x_dtype == 1 ? 4 : 8);
      void* xb = al.get<uint8_t>(bytes);
      HIPCHK(hipMemcpyAsync(xb, X, bytes, hipMemcpyHostToDevice, f.s));
      d.X = xb;
    } else {
      d.X = X;
    }
    Dev* dd = al.get<Dev>(1);
    HIPCHK(hipMemcpyAsync(dd, &d, sizeof(Dev), hipMemcpyHostToDevice, f.s));
    std::vector<int32_t> iota((size_t)p);
    for (int64_t k = 0; k < p; ++k) iota[(size_t)k] = (int32_t)k;
    init_set(d, o, limit, f.s, iota);
    Ctl c0;
    std::memset(&c0, 0, sizeof(c0));
    c0.halt_iter = -1;
    c0.root = -1;
    c0.bad_i = c0.bad_j = -1;
    HIPCHK(hipMemcpyAsync(ctl, &c0, sizeof(Ctl), hipMemcpyHostToDevice, f.s));
    HIPCHK(hipStreamSynchronize(f.s));  // host temporaries (d, iota, c0) are no longer needed

    f.b.dd = dd;
    f.b.count = 1;
    f.b.one = d;
    f.b.p_max = (int)p;
    f.b.n_max = n;
    f.b.nchunk_max = d.nchunk;
    f.b.gram_slices_max = GRAM_SLICES_MAX;
    f.b.mixed = mixed ? 1 : 0;

    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, f.s));
    // a1 + a2: normalise once, covariance once (Alg. 3)
    HIPCHK(launch_standardize(f.b, f.s));
    HIPCHK(launch_gram(f.b, 0, 0, f.s));
    Ctl c = f.drive_one(ctl, 0, limit, (int)p);
    HIPCHK(hipEventRecord(ev1, f.s));
    copy_results(d, c, n, out, f.s);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) out->seconds_device = ms * 1e-3;
    if (timer.on) {
      out->seconds_pair_kernel = timer.total_seconds();
      out->pair_kernel_launches = timer.launches;
    }
    st = (lingam_status)out->status;
    if (st != LINGAM_OK) set_error_text(st, out);
  } catch (const HipFail& e) {
    st = status_from(e);
    out->status = st;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  out->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  return st;
}

lingam_status lingam_fit_order_batch(int32_t count, const lingam_dataset* sets, const lingam_opts* opts,
                                     lingam_result* outs) {
  const auto wall0 = std::chrono::steady_clock::now();
  g_last_error.clear();
  lingam_opts o;
  if (opts) o = *opts; else lingam_opts_default(&o);
  if (count < 1 || !sets || !outs) return fail(LINGAM_E_INVALID, "empty batch or NULL arrays");
  if (count > 65535) return fail(LINGAM_E_INVALID, "at most 65535 data sets per batch");
  lingam_status st = validate_opts(o);
  if (st != LINGAM_OK) return st;
  if (o.forced_len > 0 || o.record_M_iters > 0)
    return fail(LINGAM_E_UNSUPPORTED, "forced_order and record_M_iters are not available in batches");
  for (int k = 0; k < count; ++k) {
    const lingam_dataset& ds = sets[k];
    if (!ds.X) return fail(LINGAM_E_INVALID, "data set with X == NULL");
    if (!outs[k].order) return fail(LINGAM_E_INVALID, "result->order is NULL");
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
  for (int k = 0; k < count; ++k) reset_result(&outs[k], sets[k].p, 0);

  Allocs al;
  OwnedStream os;
  PairTimer timer;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  try {
    if (o.device >= 0) HIPCHK(hipSetDevice(o.device));
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
                      : (o.precision == LINGAM_PREC_MIXED ? REFRESH_MIXED : 1);
    const bool mixed = o.precision == LINGAM_PREC_MIXED;
    f.threshold = o.use_threshold != 0;
    f.gamma0 = o.gamma0 > 0 ? o.gamma0 : 0.0;
    f.gmult = o.gamma_mult > 1.0 ? o.gamma_mult : 4.0;
    int64_t p_max = 0, n_max = 0;
    for (int k = 0; k < count; ++k) {
      p_max = std::max(p_max, sets[k].p);
      n_max = std::max(n_max, sets[k].sample_idx ? sets[k].n_idx : sets[k].n);
    }
    f.pl = make_plan(n_max, o, false);  // the chunk length is the same for every data set
    Ctl* ctls = al.get<Ctl>((size_t)count);
    std::vector<Dev> devs((size_t)count);
    f.ps.resize((size_t)count);
    f.limits.resize((size_t)count);
    // bases of bootstrap sets are uploaded once each
    std::vector<std::pair<const void*, const double*>> bases;
    std::vector<int32_t> iota((size_t)p_max);
    for (int64_t k = 0; k < p_max; ++k) iota[(size_t)k] = (int32_t)k;
    int nchunk_max = 1;
    for (int k = 0; k < count; ++k) {
      const lingam_dataset& ds = sets[k];
      const int64_t nk = ds.sample_idx ? ds.n_idx : ds.n, pk = ds.p;
      const int limit = (o.max_roots > 0 && o.max_roots < pk) ? o.max_roots : (int)pk;
      Dev d = alloc_set(al, nk, pk, f.pl, o, mixed, ctls + k);
      d.limit = limit;
      if (ds.sample_idx) {
        const double* base = nullptr;
        for (auto& bp : bases) if (bp.first == ds.X) base = bp.second;
        if (!base) {
          if (o.x_on_device) {
            base = (const double*)ds.X;
          } else {
            double* xb = al.get<double>((size_t)pk * (size_t)ds.n);
            HIPCHK(hipMemcpyAsync(xb, ds.X, sizeof(double) * pk * ds.n, hipMemcpyHostToDevice, f.s));
            base = xb;
          }
          bases.push_back({ds.X, base});
        }
        int64_t* idx_dev = al.get<int64_t>((size_t)ds.n_idx);
        HIPCHK(hipMemcpyAsync(idx_dev, ds.sample_idx, sizeof(int64_t) * ds.n_idx, hipMemcpyHostToDevice, f.s));
        double* xg = al.get<double>((size_t)pk * (size_t)nk);
        HIPCHK(launch_gather(base, ds.n, pk, idx_dev, nk, xg, f.s));
        d.X = xg;
        d.x_dtype = 0;
        d.layout = 0;
      } else if (!o.x_on_device) {
        const size_t bytes = (size_t)pk * (size_t)nk * (o.x_dtype == 1 ? 4 : 8);
        void* xb = al.get<uint8_t>(bytes);
        HIPCHK(hipMemcpyAsync(xb, ds.X, bytes, hipMemcpyHostToDevice, f.s));
        d.X = xb;
      } else {
        d.X = ds.X;
      }
      init_set(d, o, limit, f.s, iota);
      devs[(size_t)k] = d;
      f.ps[(size_t)k] = pk;
      f.limits[(size_t)k] = limit;
      nchunk_max = std::max(nchunk_max, d.nchunk);
    }
    Dev* dd = al.get<Dev>((size_t)count);
    HIPCHK(hipMemcpyAsync(dd, devs.data(), sizeof(Dev) * count, hipMemcpyHostToDevice, f.s));
    std::vector<Ctl> c0((size_t)count);
    std::memset(c0.data(), 0, sizeof(Ctl) * count);
    for (auto& c : c0) {
      c.halt_iter = -1;
      c.root = -1;
      c.bad_i = c.bad_j = -1;
    }
    HIPCHK(hipMemcpyAsync(ctls, c0.data(), sizeof(Ctl) * count, hipMemcpyHostToDevice, f.s));
    HIPCHK(hipStreamSynchronize(f.s));

    f.b.dd = dd;
    f.b.count = count;
    f.b.p_max = (int)p_max;
    f.b.n_max = n_max;
    f.b.nchunk_max = nchunk_max;
    f.b.gram_slices_max = GRAM_SLICES_MAX;
    f.b.mixed = mixed ? 1 : 0;
    int limit_max = 0;
    for (int l : f.limits) limit_max = std::max(limit_max, l);

    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, f.s));
    HIPCHK(launch_standardize(f.b, f.s));
    HIPCHK(launch_gram(f.b, 0, 0, f.s));
    // every data set steps through its iterations together; one that halts
    // (not enough threshold rounds queued, or an error) sits out from then on
    std::vector<Ctl> cs((size_t)count);
    for (int t = 0; t < limit_max;) {
      for (int q = 0; q < SYNC_EVERY && t < limit_max; ++q, ++t) f.queue_iteration(t);
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
    HIPCHK(hipMemcpyAsync(cs.data(), ctls, sizeof(Ctl) * count, hipMemcpyDeviceToHost, f.s));
    HIPCHK(hipStreamSynchronize(f.s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    st = LINGAM_OK;
    for (int k = 0; k < count; ++k) {
      copy_results(devs[(size_t)k], cs[(size_t)k], devs[(size_t)k].n, &outs[k], f.s);
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
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  for (int k = 0; k < count; ++k) outs[k].seconds_total = wall;
  return st;
}

}  // extern "C"
