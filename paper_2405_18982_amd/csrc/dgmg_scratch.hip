// Library-wide device scratch array of dgmg_vcycle_noalloc: the coarse-level
// vectors of a V-cycle for callers that cannot allocate device memory.
//
// The array is a file-scope device variable, so each GPU holds its own copy
// (allocated when the code object is loaded on that device, kept until the
// process ends).  Host code never uses the array's name as an address: the
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and cached here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dgmg_scratch.h"

namespace {

static __device__ __align__(256) unsigned char scratch[dgmg::kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace dgmg {

hipError_t scratch_address(void** ptr) {
  *ptr = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace dgmg
