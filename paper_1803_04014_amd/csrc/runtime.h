// runtime.h -- host runtime pieces shared by capi.cpp and serve.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>

namespace mfg {

// Exclusive use of the per-(device, stream) workspace for one call: holds
// the region's lock until destroyed, so two threads enqueueing on the same
// stream cannot interleave their conversions into one buffer.
class WsLease {
   public:
    WsLease(hipStream_t s, size_t bytes);
    void* ptr() const { return ptr_; }
    int status() const { return status_; }

   private:
    std::unique_lock<std::mutex> lock_;
    void* ptr_ = nullptr;
    int status_ = 0;
};

// Fault injection for tests of failure handling (MFG_FAULT=launch:<n>,alloc:<n>
// or mfg_fault_inject): the n-th kernel launch / device allocation after
// arming fails as if the HIP runtime had refused it, once.  Launches are
// counted where a GEMM, grouped or conversion launch is about to be
// enqueued, allocations where the library or the server allocates device
// memory.  Off unless armed.
enum { kFaultLaunch = 0, kFaultAlloc = 1, kFaultKinds = 2 };
void fault_arm(int64_t launch_n, int64_t alloc_n);
void fault_reload();  // re-read MFG_FAULT
bool fault_hit(int kind);
// MFG_LOG set (not "0"): one line per GEMM launch decision on stderr.
bool log_enabled();

int size_bucket(int64_t x);
int tuned_lookup(int mode, int64_t M, int64_t N, int64_t K);
void tuned_store(int mode, int64_t M, int64_t N, int64_t K, int cfg);

}  // namespace mfg
