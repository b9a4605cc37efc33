// Fixed device scratch for the entry point that allocates nothing
// (slg_components_noalloc, for callers that cannot allocate: code under
// HIP-graph capture, tight serving loops, harnesses that forbid it).
//
// The array below exists once on every GPU the library's code object is
// loaded on, from load until the process ends. Host code never uses its
// name as an address: the name is a host-side stand-in. Its device address
// is looked up per device with hipGetSymbolAddress, once, with that device
// current, and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "slg_internal.h"

static_assert(slg::kNoAllocRows % 2 == 0, "parents are packed two per int64 word");

// [0..1]: root count and error flags (int64); then one int32 union-find
// parent per hyperedge, for up to kNoAllocRows hyperedges.
static __device__ __align__(256) int64_t scratch[2 + slg::kNoAllocRows / 2];

namespace slg {

namespace {
std::mutex g_mu;
std::vector<void *> g_addr;  // per device: the array's device address (null until looked up)
}  // namespace

hipError_t noalloc_scratch(int device, void **out) {
    *out = nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device < g_addr.size() && g_addr[device]) {
        *out = g_addr[device];
        return hipSuccess;
    }
    int current = -1;
    hipError_t e = hipGetDevice(&current);
    if (e != hipSuccess) return e;
    if (current != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    if ((size_t)device >= g_addr.size()) g_addr.resize((size_t)device + 1, nullptr);
    g_addr[device] = ptr;
    *out = ptr;
    return hipSuccess;
}

}  // namespace slg
