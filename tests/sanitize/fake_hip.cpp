// Host stand-in for the HIP runtime and for the library's kernel launchers,
// so that the host side of liblingam (argument checks, workspace sizing and
// carving, the iteration loop, batch scheduling, graph cache, result copies)
// can be built with g++ and run under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.
//
// "Device" memory is host memory: hipMalloc is aligned_alloc, copies are
// memcpy, the fill launchers fill, and every other launcher returns success
// without touching memory, so the control blocks keep the state the host
// wrote (every iteration then looks finished to the host loop).
//
// Fault injection: FAKE_HIP_FAIL_MALLOC=k makes the k-th hipMalloc of the
// process (1-based) fail with hipErrorOutOfMemory; fake_hip_fail_malloc_at()
// sets the same from the test program.
#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>

#include "lingam_internal.h"

namespace {
long g_malloc_calls = 0;
long g_fail_at = -1;
int g_device = 0;
struct FakeObj { int kind; };
}  // namespace

extern "C" void fake_hip_fail_malloc_at(long k) {
  g_malloc_calls = 0;
  g_fail_at = k;
}

hipError_t hipMalloc(void** ptr, size_t size) {
  if (!ptr) return hipErrorInvalidValue;
  ++g_malloc_calls;
  if (g_fail_at < 0) {
    const char* e = std::getenv("FAKE_HIP_FAIL_MALLOC");
    g_fail_at = e ? std::atol(e) : 0;
  }
  if (g_fail_at > 0 && g_malloc_calls == g_fail_at) {
    *ptr = nullptr;
    return hipErrorOutOfMemory;
  }
  const size_t sz = (size + 255) / 256 * 256;
  *ptr = std::aligned_alloc(256, sz == 0 ? 256 : sz);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipFree(void* ptr) {
  std::free(ptr);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  if (bytes && (!dst || !src)) return hipErrorInvalidValue;
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}

hipError_t hipGetDevice(int* d) {
  if (!d) return hipErrorInvalidValue;
  *d = g_device;
  return hipSuccess;
}

hipError_t hipSetDevice(int d) {
  if (d != 0) return hipErrorInvalidDevice;
  g_device = d;
  return hipSuccess;
}

const char* hipGetErrorString(hipError_t e) {
  switch (e) {
    case hipSuccess: return "no error (fake)";
    case hipErrorOutOfMemory: return "out of memory (fake)";
    case hipErrorInvalidDevice: return "invalid device (fake)";
    default: return "error (fake)";
  }
}

hipError_t hipStreamCreate(hipStream_t* s) {
  *s = reinterpret_cast<hipStream_t>(new FakeObj{1});
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<FakeObj*>(s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(new FakeObj{2});
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<FakeObj*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (!ms || !a || !b) return hipErrorInvalidValue;
  *ms = 0.0f;
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = reinterpret_cast<hipGraph_t>(new FakeObj{3});
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  *x = reinterpret_cast<hipGraphExec_t>(new FakeObj{4});
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) { return x ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete reinterpret_cast<FakeObj*>(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete reinterpret_cast<FakeObj*>(x);
  return hipSuccess;
}

namespace lingam {

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t) {
  for (int64_t k = 0; k < count; ++k) p[k] = v;
  return hipSuccess;
}
hipError_t launch_fill_u8(uint8_t* p, int64_t count, uint8_t v, hipStream_t) {
  if (count > 0) std::memset(p, v, (size_t)count);
  return hipSuccess;
}
hipError_t launch_gather(const double* X, int64_t n_src, int64_t p, const int64_t* idx, int64_t n_idx,
                         double* out, hipStream_t) {
  // idx is read from "device" memory, as the kernel reads it; an index out
  // of range gives NaN, as in the kernel
  for (int64_t i = 0; i < p; ++i)
    for (int64_t k = 0; k < n_idx; ++k) {
      const int64_t s = idx[k];
      out[i * n_idx + k] = (s >= 0 && s < n_src) ? X[i * n_src + s] : __builtin_nan("");
    }
  return hipSuccess;
}
// initial contents and counter sums, as the device kernels set them
static void init_one(const Dev& d) {
  const int64_t P = d.p, pp = P * P;
  const double nan = __builtin_nan("");
  for (int64_t e = 0; e < pp; ++e) {
    d.M[e] = d.Tall[e] = d.Hall[e] = d.Terr[e] = d.Terrp[e] = nan;
    d.Tstate[e] = 0;
    d.pend[e] = 0;
  }
  if (d.Mrec)
    for (int64_t e = 0; e < (int64_t)d.rec * pp; ++e) d.Mrec[e] = nan;
  for (int64_t i = 0; i < P; ++i) {
    d.idx[0][i] = d.ord[0][i] = (int32_t)i;
    d.order[i] = -1;
  }
  for (int e = 0; e < 2 * PAIR_SLOTS; ++e) d.pair_slots[e] = 0;
  Ctl c{};
  c.halt_iter = -1;
  c.root = -1;
  c.bad_i = c.bad_j = -1;
  *d.ctl = c;
}
hipError_t launch_init_sets(const Batch& b, hipStream_t) {
  for (int k = 0; k < b.count; ++k) init_one(b.count == 1 ? b.one : b.dd[k]);
  return hipSuccess;
}
hipError_t launch_sum_slots(const Batch& b, hipStream_t) {
  for (int k = 0; k < b.count; ++k) {
    const Dev& d = b.count == 1 ? b.one : b.dd[k];
    unsigned long long ev = 0, comp = 0;
    for (int i = 0; i < PAIR_SLOTS; ++i) {
      ev += d.pair_slots[i];
      comp += d.pair_slots[PAIR_SLOTS + i];
    }
    d.pair_slots[0] = ev;
    d.pair_slots[1] = comp;
  }
  return hipSuccess;
}
hipError_t launch_standardize(const Batch&, hipStream_t) { return hipSuccess; }
hipError_t launch_gram(const Batch&, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_iter_start(const Batch&, int, double, double, int, int, hipStream_t) { return hipSuccess; }
void pair_band_shape(const Batch&, int& rows_per_group, int& groups) {
  rows_per_group = 2;
  groups = 1024;
}
hipError_t launch_pair_band(const Batch&, int, const BandArgs&, int, int, hipStream_t, hipEvent_t, hipEvent_t) {
  return hipSuccess;
}
hipError_t launch_pair_baseline(const Batch&, int, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_score(const Batch&, int, const BandArgs&, double, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_window_reset(const Batch&, hipStream_t) { return hipSuccess; }
hipError_t launch_record_M(const Batch&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_iter_end(const Batch&, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_last(const Batch&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_resume(const Batch&, hipStream_t) { return hipSuccess; }
hipError_t launch_term_sweep(TermSweep* out, hipStream_t) {
  std::memset(static_cast<void*>(out), 0, sizeof(TermSweep));
  return hipSuccess;
}
hipError_t launch_corr_snapshot(const Dev&, hipStream_t) { return hipSuccess; }
hipError_t launch_estimate_B(const Dev&, hipStream_t) { return hipSuccess; }

}  // namespace lingam
