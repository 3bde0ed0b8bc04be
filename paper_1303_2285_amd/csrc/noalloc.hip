// noalloc.hip -- the fixed device scratch of covest_forward_noalloc.
//
// One file-scope device array holds everything the recurrence needs beyond A
// and R: the plan's job tables and the FP64 workspace.  Each device that runs
// the library holds its own copy until the process ends.  In host code the
// array's name is not a device address, so the address is looked up once per
// device (with that device current) and only that pointer is handed out.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "noalloc_internal.hpp"

static __device__ __align__(256) unsigned char scratch[covest::kNoallocScratchBytes];

namespace {
std::mutex g_mu;
std::map<int, void *> g_scratch;   // device -> address of its copy of `scratch`
}  // namespace

namespace covest {

hipError_t noalloc_scratch(void **out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch.emplace(dev, p);
    *out = p;
    return hipSuccess;
}

}  // namespace covest
