// Fixed device scratch for the allocation-free merge entry point
// (xrd_merge_peaks_noalloc): a file-scope device array of kNoallocBytes that
// every GPU the library runs on holds until the process ends.
//
// In host code the array's name is only a host-side stand-in, not a device
// address, so the host never passes it anywhere: on the first call on a
// device (with that device current) its device address is taken with
// hipGetSymbolAddress and kept per device, and only that address reaches
// kernels and copies.  Each device holds its own copy of the array at its own
// address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "xrd_internal.h"

namespace xrd {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(void **out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || reinterpret_cast<uintptr_t>(p) % 256) return hipErrorInvalidValue;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace xrd
