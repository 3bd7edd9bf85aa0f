// Library-owned exchange buffer of moff_correlate_noalloc, for callers that cannot allocate device memory.
//
// The buffer is a file-scope device array: each GPU the library runs on holds its own copy, at its own address,
// from the first call on that device until the process ends.  In host code the array's name is only a host-side
// stand-in, so its device address is looked up once per device (with that device current) and kept; kernels get
// that address as an argument, like the workspace's exchange region.  Every call on one GPU shares the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "kernels.h"

namespace moff {

static __device__ __align__(256) float2 scratch[kNoallocExchangeBytes / sizeof(float2)];

hipError_t noalloc_exchange(void **ptr, size_t *bytes) {
  static std::mutex mu;
  static std::vector<void *> per_device;   // device address of `scratch` on each device, once looked up
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if ((size_t)dev >= per_device.size()) per_device.resize((size_t)dev + 1, nullptr);
  if (!per_device[(size_t)dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[(size_t)dev] = p;
  }
  *ptr = per_device[(size_t)dev];
  *bytes = kNoallocExchangeBytes;
  return hipSuccess;
}

}  // namespace moff
