// Static device scratch of the allocation-free product (dh2_matvec_noalloc):
// one array per GPU, part of the library's code object, allocated when the
// library is loaded on a device and held until the process ends.  Host code
// never names the array except in the address lookup below: on the host its
// name is only a stand-in, and a kernel handed that stand-in would fault.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "scratch.hpp"

namespace dh2 {

static __device__ __align__(256) char scratch[kScratchBytes];

void* scratch_region(size_t* bytes) {
  static std::mutex mu;
  static std::map<int, void*> addr;   // device -> address of its copy (nullptr: lookup failed)
  if (bytes) *bytes = kScratchBytes;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    it = addr.emplace(dev, p).first;
  }
  return it->second;
}

}  // namespace dh2
