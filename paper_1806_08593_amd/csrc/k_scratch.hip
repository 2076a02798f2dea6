// Device-resident workspace of the allocation-free forward entry point
// (tmc_gauss_fwd_noalloc): one file-scope device array, which every GPU the library
// runs on holds at its own address until the process ends.  In host code the array's
// name is only a host-side stand-in; its device address on a GPU comes from
// hipGetSymbolAddress, taken once per device at plan creation (that device current)
// and kept per device here.  Kernels are only ever given that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tmc_scratch.h"

namespace tmc {

static __device__ __align__(256) unsigned char scratch[kNoallocWorkspaceBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* scratch_device_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace tmc
