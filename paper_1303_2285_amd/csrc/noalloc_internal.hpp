// noalloc_internal.hpp -- the fixed device scratch behind covest_forward_noalloc.
#pragma once

#include <cstddef>

#include <hip/hip_runtime_api.h>

#include "covest.h"

namespace covest {

constexpr size_t kNoallocScratchBytes = COVEST_NOALLOC_SCRATCH_BYTES;

// Device address of the current device's scratch array (looked up on the
// first call for each device, then cached).
hipError_t noalloc_scratch(void **out);

}  // namespace covest
