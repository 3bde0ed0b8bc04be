// device_util.hpp -- small device helpers shared by the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

namespace covest {

// Workgroup b of a launch runs on XCD b % 8.  Map the workgroups of one XCD
// to one contiguous range of the work list (any n), so that neighbouring work
// items (jobs over one region of A, or finalize items of neighbouring lags,
// whose partial sums share cache lines) meet in the same L2.
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int x = b & 7;
    return x * (n >> 3) + min(x, n & 7) + (b >> 3);
}

}  // namespace covest
