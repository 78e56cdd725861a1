// Drives every entry point of liblingam's host side (built against the
// host stand-in of fake_hip.cpp) through valid calls, argument errors,
// undersized workspaces and failed allocations.  Run under ASan/UBSan: any
// sanitizer report aborts the program; a wrong status prints and exits 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lingam.h"

extern "C" void fake_hip_fail_malloc_at(long k);

static int g_fail = 0;

static void expect(lingam_status got, lingam_status want, const char* what) {
  if (got != want) {
    std::printf("FAIL %s: status %d (%s), expected %d; last error: %s\n", what, (int)got,
                lingam_status_string(got), (int)want, lingam_last_error());
    g_fail = 1;
  }
}

struct Out {
  std::vector<int32_t> order;
  std::vector<double> T, H, M, Eb, Ep, B;
  std::vector<uint8_t> S;
  lingam_result r;
  Out(int64_t p, int rec = 0, bool all = true) : order(p), T(p * p), H(p * p), M(rec * p * p + 1),
      Eb(p * p), Ep(p * p), B(p * p), S(p * p) {
    std::memset(&r, 0, sizeof r);
    r.order = order.data();
    if (all) {
      r.T = T.data(); r.H = H.data(); r.T_state = S.data(); r.T_err_bound = Eb.data();
      r.T_err_prob = Ep.data(); r.B = B.data();
      if (rec) r.M = M.data();
    }
  }
};

static std::vector<double> data(int64_t p, int64_t n, unsigned seed) {
  std::vector<double> x(p * n);
  uint64_t s = 0x9E3779B97F4A7C15ull * (seed + 1);
  for (auto& v : x) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    v = (double)(s >> 11) * 0x1.0p-53 - 0.5;
  }
  return x;
}

int main() {
  lingam_opts o;
  lingam_opts_default(&o);
  for (int s = 0; s <= 7; ++s) (void)lingam_status_string((lingam_status)s);
  (void)lingam_last_error();

  // valid searches in every precision, input form and option set
  const int64_t shapes[][2] = {{1, 16}, {2, 5}, {9, 700}, {40, 3001}};
  for (auto& sh : shapes) {
    const int64_t p = sh[0], n = sh[1];
    auto X = data(p, n, (unsigned)(p + n));
    std::vector<float> Xf(X.begin(), X.end());
    for (int prec = 0; prec <= 2; ++prec)
      for (int variant = 0; variant < 6; ++variant) {
        lingam_opts q = o;
        q.precision = prec;
        q.record_M_iters = variant == 1 ? (int32_t)(p < 3 ? p : 3) : 0;
        q.use_threshold = variant != 2;
        q.messaging = variant != 3;
        q.layout = variant == 4 ? LINGAM_LAYOUT_SAMPLE_MAJOR : LINGAM_LAYOUT_VAR_MAJOR;
        q.x_dtype = variant == 5 ? 1 : 0;
        q.x_on_device = variant == 5;
        q.estimate_B = variant == 0;
        q.profile = variant == 1;
        q.max_roots = variant == 2 ? (int32_t)(p / 2) : 0;
        q.chunk_samples = variant == 3 ? 256 : 0;
        Out out(p, q.record_M_iters);
        const void* src = q.x_dtype ? (const void*)Xf.data() : (const void*)X.data();
        expect(lingam_fit_order(src, n, p, &q, &out.r), LINGAM_OK, "fit_order");
        // the same call on a caller workspace, exactly sized and one byte short
        const uint64_t need = lingam_workspace_size(n, p, &q);
        void* ws = std::aligned_alloc(256, (need + 255) / 256 * 256);
        q.workspace = ws;
        q.workspace_bytes = need;
        if (!q.profile) expect(lingam_fit_order(src, n, p, &q, &out.r), LINGAM_OK, "fit_order workspace");
        q.workspace_bytes = need - 1;
        if (!q.profile) expect(lingam_fit_order(src, n, p, &q, &out.r), LINGAM_E_NOMEM, "short workspace");
        q.workspace = static_cast<char*>(ws) + 8;
        q.workspace_bytes = need;
        expect(lingam_fit_order(src, n, p, &q, &out.r), LINGAM_E_INVALID, "misaligned workspace");
        std::free(ws);
      }
    // the baseline pair strategies (FP64, no threshold, no messaging), and
    // the combinations they refuse
    for (int strategy = LINGAM_PAIR_BLOCK_WORKER; strategy <= LINGAM_PAIR_BLOCK_COMPARE; ++strategy) {
      lingam_opts q = o;
      q.pair_strategy = strategy;
      q.use_threshold = 0;
      q.messaging = 0;
      Out out(p, 0);
      expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_OK, "baseline strategy");
      q.use_threshold = 1;
      expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "baseline with threshold");
      q.use_threshold = 0;
      q.precision = LINGAM_PREC_MIXED;
      expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "baseline in mixed precision");
    }
    {
      lingam_opts q = o;
      q.pair_strategy = 4;
      Out out(p, 0);
      expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "unknown strategy");
    }
    // step 2 on its own
    std::vector<int32_t> ord(p);
    for (int64_t k = 0; k < p; ++k) ord[k] = (int32_t)(p - 1 - k);
    std::vector<double> B(p * p);
    expect(lingam_estimate_B(X.data(), n, p, ord.data(), &o, B.data()), LINGAM_OK, "estimate_B");
    if (p > 1) {
      ord[0] = ord[1];
      expect(lingam_estimate_B(X.data(), n, p, ord.data(), &o, B.data()), LINGAM_E_INVALID, "estimate_B bad order");
    }
  }

  // forced prefix
  {
    const int64_t p = 9, n = 300;
    auto X = data(p, n, 7);
    const int32_t pre[3] = {4, 0, 8};
    lingam_opts q = o;
    q.forced_order = pre;
    q.forced_len = 3;
    Out out(p);
    expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_OK, "forced prefix");
    const int32_t bad[2] = {4, 4};
    q.forced_order = bad;
    q.forced_len = 2;
    expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "forced duplicate");
    const int32_t oob[1] = {9};
    q.forced_order = oob;
    q.forced_len = 1;
    expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "forced out of range");
  }

  // argument errors
  {
    const int64_t p = 5, n = 64;
    auto X = data(p, n, 3);
    Out out(p);
    expect(lingam_fit_order(nullptr, n, p, &o, &out.r), LINGAM_E_INVALID, "null X");
    expect(lingam_fit_order(X.data(), 1, p, &o, &out.r), LINGAM_E_INVALID, "n = 1");
    expect(lingam_fit_order(X.data(), n, 0, &o, &out.r), LINGAM_E_INVALID, "p = 0");
    expect(lingam_fit_order(X.data(), n, p, nullptr, &out.r), LINGAM_OK, "default opts");
    lingam_opts q = o;
    q.struct_size = 8;
    expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "struct_size");
    q = o;
    q.precision = 7;
    expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "precision");
    q = o;
    q.chunk_samples = 100;
    expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_INVALID, "chunk_samples");
    q = o;
    q.device = 3;
    expect(lingam_fit_order(X.data(), n, p, &q, &out.r), LINGAM_E_DEVICE, "device 3");
    lingam_result r0 = out.r;
    r0.order = nullptr;
    expect(lingam_fit_order(X.data(), n, p, &o, &r0), LINGAM_E_INVALID, "null order");
    if (lingam_workspace_size(n, 0, &o) != 0 || lingam_workspace_size(1, p, &o) != 0) {
      std::printf("FAIL workspace_size of an invalid shape is not 0\n");
      g_fail = 1;
    }
    // a failed allocation is NOMEM and leaves nothing behind
    fake_hip_fail_malloc_at(1);
    expect(lingam_fit_order(X.data(), n, p, &o, &out.r), LINGAM_E_NOMEM, "failed allocation");
    fake_hip_fail_malloc_at(0);
    // a non-finite input is caught on the host for host inputs only when the
    // device reports it; with the stand-in the search completes
    expect(lingam_fit_order(X.data(), n, p, &o, &out.r), LINGAM_OK, "after failed allocation");
  }

  // batches: own data, bootstrap resamples, uneven shapes; queue, slices, graphs
  {
    const int count = 7;
    std::vector<std::vector<double>> Xs;
    std::vector<lingam_dataset> sets(count);
    auto base = data(12, 500, 11);
    std::vector<std::vector<int64_t>> idx;
    for (int k = 0; k < count; ++k) {
      const int64_t p = 3 + 5 * k, n = 200 + 97 * k;
      Xs.push_back(data(p, n, 20 + k));
      sets[k] = {Xs.back().data(), n, p, nullptr, 0};
      if (k % 3 == 2) {
        idx.emplace_back(450 + k);
        for (size_t j = 0; j < idx.back().size(); ++j) idx.back()[j] = (int64_t)((j * 7919) % 500);
        sets[k] = {base.data(), 500, 12, idx.back().data(), (int64_t)idx.back().size()};
      }
    }
    for (int prec = 0; prec <= 2; ++prec)
      for (int mode = 0; mode < 4; ++mode) {
        lingam_opts q = o;
        q.precision = prec;
        q.batch_queue = mode != 1;
        q.max_roots = mode == 3 ? 2 : 0;
        std::vector<Out> outs;
        std::vector<lingam_result> rs;
        for (int k = 0; k < count; ++k) outs.emplace_back(sets[k].p, 0, true);
        for (auto& x : outs) { x.r.B = nullptr; rs.push_back(x.r); }
        void* ws = nullptr;
        if (mode == 2) {
          q.graph = 1;
          const uint64_t need = lingam_workspace_size_batch(count, sets.data(), &q);
          ws = std::aligned_alloc(256, (need + 255) / 256 * 256);
          q.workspace = ws;
          q.workspace_bytes = need;
        }
        for (int rep = 0; rep < (mode == 2 ? 3 : 1); ++rep)
          expect(lingam_fit_order_batch(count, sets.data(), &q, rs.data()), LINGAM_OK, "batch");
        if (ws) {
          q.workspace_bytes -= 256;
          expect(lingam_fit_order_batch(count, sets.data(), &q, rs.data()), LINGAM_E_NOMEM, "batch short workspace");
          std::free(ws);
        }
      }
    lingam_opts q = o;
    q.record_M_iters = 1;
    std::vector<lingam_result> rs(count);
    std::vector<Out> outs;
    for (int k = 0; k < count; ++k) { outs.emplace_back(sets[k].p, 0, false); rs[k] = outs.back().r; }
    expect(lingam_fit_order_batch(count, sets.data(), &q, rs.data()), LINGAM_E_UNSUPPORTED, "batch record_M");
    q = o;
    q.pair_strategy = LINGAM_PAIR_BLOCK_COMPARE;
    q.use_threshold = 0;
    q.messaging = 0;
    expect(lingam_fit_order_batch(count, sets.data(), &q, rs.data()), LINGAM_E_UNSUPPORTED, "batch baseline strategy");
    expect(lingam_fit_order_batch(0, sets.data(), &o, rs.data()), LINGAM_E_INVALID, "batch of 0");
    std::vector<int64_t> badidx = {0, 1, 500};
    lingam_dataset bad = {base.data(), 500, 12, badidx.data(), 3};
    expect(lingam_fit_order_batch(1, &bad, &o, rs.data()), LINGAM_E_INVALID, "bootstrap index out of range");
  }

  // the hardware term sweep (zeros from the stand-in)
  {
    lingam_term_check tc;
    expect(lingam_check_terms(-1, &tc), LINGAM_OK, "check_terms");
    expect(lingam_check_terms(-1, nullptr), LINGAM_E_INVALID, "check_terms null");
  }

  std::printf(g_fail ? "driver host checks FAILED\n" : "driver host checks passed\n");
  return g_fail;
}
