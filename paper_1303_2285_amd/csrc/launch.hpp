// launch.hpp -- host entry points of the HIP kernels (one per kernel file).
#pragma once

#include <hip/hip_runtime.h>

#include "covest_internal.hpp"

namespace covest {

// Sets the dynamic-LDS limits of every recurrence kernel (call before graph capture).
hipError_t prepare_rec_kernels();
hipError_t launch_rec_main(const MainArgs &ma, int n_blocks, size_t lds_bytes, hipStream_t stream);
hipError_t launch_rec_persistent(const MainArgs &ma, unsigned int *counter, int n_blocks, size_t lds_bytes,
                                 hipStream_t stream);
// variant: kFinTable, kFinTableSmall (plan.hpp) or kFinLean
hipError_t launch_rec_finalize(const FinArgs &fa, int n_blocks, size_t lds_bytes, int variant,
                               hipStream_t stream);

// Matrix-core main pass (rec_mfma.hip): mt x nt tiles of the orientation-0 lag block.
hipError_t launch_rec_mfma(const MfmaArgs &ma, int mt, int nt, int n_blocks, size_t lds, hipStream_t stream);

}  // namespace covest
