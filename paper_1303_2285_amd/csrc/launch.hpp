// launch.hpp -- host entry points of the HIP kernels (one per kernel file).
#pragma once

#include <hip/hip_runtime.h>

#include "covest_internal.hpp"

namespace covest {

hipError_t launch_rec_main(const MainArgs &ma, int n_blocks, size_t lds_bytes, hipStream_t stream);
hipError_t launch_rec_finalize(const FinArgs &fa, int n_blocks, size_t lds_bytes, bool table,
                               hipStream_t stream);

}  // namespace covest
