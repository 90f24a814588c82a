// spaqr_apply_noalloc: the preconditioner apply (Section 2.8) for callers
// that cannot allocate device memory.  Its only workspace -- the permuted
// right-hand sides the sweeps update in place -- lives in a fixed device
// array of this library instead of memory allocated per call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "engine.hpp"

namespace {

// 2^23 doubles (64 MiB) per GPU: n * nrhs of one call may not exceed it.
constexpr int64_t kScratchDoubles = int64_t(1) << 23;

// The array's name is a host-side stand-in in host code: kernels receive the
// per-device address hipGetSymbolAddress returns for it, never the name.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
std::vector<double*> g_ptr;  // address of `scratch` on each device, set once

// Address of the copy of `scratch` on the device of stream s (the current
// device for the null stream), looked up once per device with that device
// current.
double* scratch_for(hipStream_t s) {
  int cur = 0;
  SPAQR_HIP(hipGetDevice(&cur));
  int dev = cur;
  if (s) {
    hipDevice_t d = 0;
    SPAQR_HIP(hipStreamGetDevice(s, &d));
    dev = (int)d;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ptr.size() <= dev) g_ptr.resize(dev + 1, nullptr);
  if (!g_ptr[dev]) {
    if (dev != cur) SPAQR_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      throw spaqr::Error(SPAQR_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_ptr[dev] = static_cast<double*>(p);
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

spaqr_status spaqr_apply_noalloc(spaqr_handle* h, const double* b, double* x, int64_t nrhs, int64_t ld) {
  try {
    SPAQR_REQUIRE(h && h->e && b && x && nrhs >= 1 && ld >= h->e->n(), SPAQR_EINVAL, "bad argument");
    SPAQR_REQUIRE(h->e->stages_left() == 0 && h->e->error() == SPAQR_OK, SPAQR_EINVAL,
                  "the handle holds no complete factorization");
    SPAQR_REQUIRE(nrhs <= kScratchDoubles / h->e->n(), SPAQR_EINVAL,
                  "n * nrhs exceeds the 2^23 doubles of the allocation-free apply's workspace");
    double* ws = scratch_for(h->e->stream());
    h->e->apply_ws(b, ld, x, ld, (int)nrhs, ws);
    return SPAQR_OK;
  } catch (const spaqr::Error& e) {
    return e.status;
  } catch (...) {
    return SPAQR_EDEVICE;
  }
}

int64_t spaqr_apply_noalloc_max(void) { return kScratchDoubles; }

}  // extern "C"
