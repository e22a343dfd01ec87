// sf_noalloc.hip -- the fixed scratch buffer of the allocation-free entry
// point (sf_reduce_begin_noalloc): one statically sized device array per
// device, whose address is looked up once per device and then passed to the
// kernels like any other scratch pointer.
#include <mutex>

#include "sf_internal.h"

namespace sfi {

static_assert(SF_NOALLOC_SCRATCH_BYTES % 256 == 0, "fixed scratch size");

// Every device the library runs on holds its own copy until the process
// ends.  Host code never uses this name as an address: only the pointer
// returned by hipGetSymbolAddress for the current device.
static __device__ __align__(256) unsigned char scratch[SF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

int fixed_scratch(void **ptr, size_t *bytes) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_hip_error(e);
  if (dev < 0 || dev >= kMaxDevices) return SF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = SF_NOALLOC_SCRATCH_BYTES;
  return SF_OK;
}

}  // namespace sfi
