// Device memory for the allocation-free entry point (lsq_fused_pass_noalloc): the per-workgroup
// partials of the fused pass and its two reduction stages live in a file-scope device array instead of
// the context's workspace, for callers that cannot allocate device memory.
#include <mutex>

#include "internal.h"

namespace lsq {

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on device `dev`, which must be the current device.  Each device holds
// its own copy of the array at its own address; the host-side name is only a stand-in, so the address
// is looked up once per device and kept.
hipError_t noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace lsq
