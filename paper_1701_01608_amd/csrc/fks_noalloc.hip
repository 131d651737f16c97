// Library-owned scratch for callers that cannot allocate device memory (code under
// stream capture, serving loops): a file-scope device array of fixed size.  Each GPU the
// library runs on holds its own copy until the process ends.  Its device address is looked
// up once per device with hipGetSymbolAddress (in host code the array's name is only a
// host-side stand-in, not a device address) and cached; every use on a device goes
// through that cached pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fks_internal.hpp"

namespace fks {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void** ptr) {
  *ptr = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace fks
