// noalloc.hip -- the fixed device scratch behind ks_keyswitch_noalloc.
//
// The array below is a device variable: every GPU the library runs on holds
// its own copy, at its own address, until the process ends.  In host code
// its name stands for a host-side shadow, not a device address, so host code
// never passes the name itself to a kernel or a copy: the device address of
// each GPU's copy is looked up once per device (hipGetSymbolAddress, with
// that device current) and kept here.
#include <mutex>

#include "kernels.h"

namespace {

static __device__ __align__(256) uint32_t scratch[KS_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

namespace ks {

hipError_t noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[dev]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != dev) return hipErrorInvalidDevice;
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p || ((uintptr_t)p & 255)) return hipErrorInvalidValue;
  g_ptr[dev] = p;
  return hipSuccess;
}

void *noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return g_ptr[dev];
}

}  // namespace ks
