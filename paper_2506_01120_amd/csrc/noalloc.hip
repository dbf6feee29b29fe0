// Fixed device workspace for the entry points that allocate nothing.
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc) use lie_closure_orthogonality_noalloc,
// whose partial Gram panels and partial sums live in the file-scope array below
// instead of a per-call allocation.  Each GPU the library runs on holds its own
// copy of the array until the process ends; its device address is looked up once
// per device, with that device current, when a handle is created on it.  In host
// code the array's name is not a device address: only the looked-up pointer is
// ever passed to a kernel or a copy.
#include "lie_internal.h"

#include <mutex>

namespace lie {

namespace {

static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device])
        return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    g_scratch[device] = static_cast<double *>(ptr);
    return hipSuccess;
}

double *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

}  // namespace lie
