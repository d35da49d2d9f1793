// lc_static.hip -- the library's static device scratch.
//
// A file-scope device array that sweeps of small chains can run in without
// any allocation (lc_update_noalloc, for callers that cannot allocate device
// memory: code under graph capture, tight serving loops).  Every GPU the
// library runs on holds its own copy of the array at its own address until
// the process ends; host code must use that address, obtained once per
// device with hipGetSymbolAddress, never the array's name (which in host code
// is only a stand-in).  All calls on one GPU share the array: calls that
// overlap on one GPU race, and nothing in it survives from one call to the
// next (every sweep clears what must start at zero).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lc_static.h"

static __device__ __align__(256) unsigned char scratch[LC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Device address of this GPU's copy of the scratch array (the current
// device), found once per device; nullptr on a HIP error.
void* lc_static_scratch(size_t* bytes) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> hold(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  if (bytes) *bytes = LC_STATIC_SCRATCH_BYTES;
  return g_ptr[dev];
}
