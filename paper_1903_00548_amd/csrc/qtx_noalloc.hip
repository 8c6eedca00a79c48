// Fixed device scratch for callers that cannot allocate device memory (code
// under graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The array lives in the library's code object, so every GPU the library
// runs on holds its own copy, allocated when the code object is loaded and
// kept until the process ends.  In host code the array's name is only a
// host-side stand-in: its device address comes from hipGetSymbolAddress,
// called once per device with that device current, and only that address
// is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qtx_internal.h"

namespace qtx {

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, char** ptr) {
  static std::mutex mu;
  static char* per_device[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!per_device[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    per_device[device] = static_cast<char*>(p);
  }
  *ptr = per_device[device];
  return hipSuccess;
}

}  // namespace qtx
