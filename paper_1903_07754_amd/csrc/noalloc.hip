// Fixed device scratch of the allocation-free BFS entry point (wedge_bfs_noalloc).
//
// Callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid hipMalloc) run BFS with this
// array as its whole workspace. It is a file-scope device array: every GPU
// the library runs on holds its own copy, at its own address, from the
// module's load until the process ends. In host code the array's name is a
// host-side stand-in, not a device address, so it is never passed to a
// kernel or a copy: the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wedge_internal.h"

namespace wedge {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_lookup_mu;
void* g_scratch[kNoAllocMaxDevices];
std::mutex g_run_mu[kNoAllocMaxDevices];

}  // namespace

hipError_t noalloc_scratch(int dev, void** ptr) {
    *ptr = nullptr;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_lookup_mu);
    if (!g_scratch[dev]) {
        SetupLock setup;  // the lookup may load the module on this device
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev) return hipErrorInvalidDevice;  // the lookup is made on the current device
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return hipSuccess;
}

std::mutex& noalloc_run_lock(int dev) { return g_run_mu[dev]; }

}  // namespace wedge
