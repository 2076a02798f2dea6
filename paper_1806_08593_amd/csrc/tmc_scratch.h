// The library's static device workspace (k_scratch.hip), used by the allocation-free
// forward entry point.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace tmc {

// Bytes of the static device workspace per GPU (must equal TMC_NOALLOC_WORKSPACE_MAX).
constexpr size_t kNoallocWorkspaceBytes = (size_t)64 << 20;
constexpr int kMaxScratchDevices = 64;

// Looks up the device address of the static workspace on `device`, which must be the
// current device; once per device (later calls return at once).  Thread-safe.
hipError_t scratch_init(int device);
// The address scratch_init found for `device`, or nullptr before it succeeded.
void* scratch_device_ptr(int device);

}  // namespace tmc
