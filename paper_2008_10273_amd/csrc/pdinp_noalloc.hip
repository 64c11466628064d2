// Static device scratch of decode_residual_batch_noalloc: the status word,
// the counters, the deferred-block list, the wave-per-block queues and the
// global-memory bordered systems of a decode live in one file-scope device
// array instead of context allocations, so that the entry point allocates
// nothing.  Every GPU the library runs on holds its own copy of the array
// (kNoAllocScratchBytes) until the process ends.
//
// In host code the array's name is only a stand-in for the device symbol:
// its device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is handed to kernels.
#include "pdinp_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace pdi {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of each device's copy (null: not set up)
}  // namespace

hipError_t noalloc_setup(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    // the status word and the counters start at zero (every decode leaves its
    // counters at zero again; the status word is cleared by pdi_sync)
    if (e == hipSuccess) e = hipMemset(p, 0, kNoAllocHeadBytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace pdi
