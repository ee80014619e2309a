// Static device scratch of the allocation-free V-cycle (definitions in noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "r3mg.h"

namespace r3mg {

// capacity of the scratch: the V-cycle work vectors of the allocation-free entry point
constexpr size_t kNoallocScratchBytes = (size_t)R3MG_NOALLOC_SCRATCH_BYTES;

// Device address of device `dev`'s scratch, looked up once per device (the device must be current at the first
// call on it); throws Error on failure.
void* scratch_device_ptr(int dev);

// zero `bytes` (rounded up to 16) at device address p with a fill kernel (no hipMemsetAsync: the call may be
// captured into a graph)
void scratch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace r3mg
