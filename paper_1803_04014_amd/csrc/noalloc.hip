// noalloc.hip -- device storage of mfg_gemm_noalloc: the operands it
// converts (rounded, split or quantised FP32 inputs) go into a fixed array
// that the code object carries, instead of a workspace grown with hipMalloc.
//
// Every device the library runs on holds its own copy of `scratch`, from the
// moment the code object is loaded on it until the process ends.  In host
// code the array's name is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, resolved once per device (with
// that device current) and kept; only that address ever reaches a kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

static __device__ __align__(256) unsigned char scratch[MFG_NOALLOC_SCRATCH_BYTES];

namespace mfg {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

// This device's copy of the array (resolved on the first call per device).
int noalloc_scratch(void** ptr, size_t* bytes) {
    int dev = 0;
    MFG_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MFG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        MFG_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return MFG_ERR_INTERNAL;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    *bytes = (size_t)MFG_NOALLOC_SCRATCH_BYTES;
    return MFG_OK;
}

}  // namespace mfg
