// Fixed device scratch of the allocation-free entry point.
//
// One file-scope array per device, alive until the process ends.  Host code
// never uses the array's name as an address: its device address is looked
// up once per device (with that device current) and cached here.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "sky_kernels.h"

namespace sky {
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(1) << 20;   // 8 MiB
}  // namespace sky

static __device__ __align__(256) double scratch[sky::NOALLOC_SCRATCH_DOUBLES];

namespace sky {

size_t noalloc_scratch_capacity() { return NOALLOC_SCRATCH_DOUBLES; }

int noalloc_scratch(double** ptr, std::string* err) {
  static std::mutex mu;
  static std::vector<double*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return -1;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (size_t(dev) >= addr.size()) addr.resize(size_t(dev) + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return -1;
    }
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return 0;
}

}  // namespace sky
