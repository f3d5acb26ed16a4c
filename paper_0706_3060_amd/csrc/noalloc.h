// Interface of the device scratch area (noalloc.hip) to the host runtime: the
// memory of the allocation-free forward entry point.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace nbk {

// Size of the scratch area each GPU holds for the process's lifetime: the
// padded j-records and the split partials of one forward evaluation.
constexpr size_t kScratchBytes = size_t(64) << 20;

// Device address of the current device's scratch area (looked up once per
// device, with that device current, and kept).
hipError_t scratch_area(void **ptr);

}  // namespace nbk
