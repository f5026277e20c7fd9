// Static device workspace of ffa_search_noalloc, the search entry point that
// allocates no device memory.
//
// The workspace is one file-scope array, so every device the library runs on
// holds its own copy of it, at its own address, from the library's first use
// on that device until the process ends. In host code the array's name only
// stands for the variable: its device address on the current device comes from
// hipGetSymbolAddress, taken once per device by ffa_create (noalloc_setup) and
// kept; kernels, copies and fills take that address, never the name.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ffa_kernels.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[ffa::kNoAllocBytes];

std::mutex g_mutex;
void* g_ptr[ffa::kMaxDevices] = {};

}  // namespace

namespace ffa {

hipError_t noalloc_setup(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace ffa
