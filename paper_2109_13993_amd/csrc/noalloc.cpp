// lingam_fit_order_noalloc: the causal-order search for callers that cannot
// allocate device memory.  Every device buffer of the call is carved from a
// fixed, file-scope device array (`scratch`) that each GPU holds for the
// life of the process; nothing is allocated per call (no device memory,
// streams or events).
#include "lingam.h"
#include "lingam_internal.h"

#include <cstdio>
#include <mutex>

namespace {

constexpr uint64_t NOALLOC_BYTES = 64ull << 20;   // 64 MiB per GPU
constexpr int NOALLOC_MAX_DEVICES = 64;

// One copy per GPU.  In host code this name is only a stand-in for the
// symbol, never a device address: the address of the current GPU's copy
// comes from hipGetSymbolAddress, and only that address reaches kernels.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void* g_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `dev`'s copy of scratch, looked up once per device with
// that device current.  Returns nullptr (and the HIP error in *err) on failure.
void* scratch_of(int dev, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    g_ptr[dev] = ptr;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" lingam_status lingam_fit_order_noalloc(const void* X, int64_t n, int64_t p, const lingam_opts* opts,
                                                  lingam_result* out) {
  lingam_opts o;
  if (opts) o = *opts; else lingam_opts_default(&o);
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) {
    lingam::set_last_error("hipGetDevice failed");
    return LINGAM_E_DEVICE;
  }
  const int dev = o.device >= 0 ? o.device : prev;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    lingam::set_last_error("device ordinal out of range for lingam_fit_order_noalloc");
    return LINGAM_E_INVALID;
  }
  if (dev != prev && hipSetDevice(dev) != hipSuccess) {
    lingam::set_last_error("hipSetDevice failed");
    return LINGAM_E_DEVICE;
  }
  hipError_t err = hipSuccess;
  void* base = scratch_of(dev, &err);
  lingam_status st;
  if (!base) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(err));
    lingam::set_last_error(buf);
    st = LINGAM_E_DEVICE;
  } else {
    const lingam::FixedBlock block{static_cast<char*>(base), NOALLOC_BYTES, "lingam_fit_order_noalloc"};
    o.device = dev;
    st = lingam::fit_order_in_block(X, n, p, &o, out, block);
  }
  if (dev != prev) (void)hipSetDevice(prev);
  return st;
}
