// Device scratch of alb_sssp_noalloc: one file-scope device array per GPU,
// loaded with this code object and held until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress (with
// that device current) and kept; host code passes that address to kernels,
// never the array's name (which on the host is only a stand-in).
#include <hip/hip_runtime.h>

#include <mutex>

#include "alb_internal.h"

static __device__ __align__(256) unsigned char scratch[alb::kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

namespace alb {

hipError_t noalloc_scratch(int device, void **ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255u)) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace alb
