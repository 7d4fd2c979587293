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

int size_bucket(int64_t x);
int tuned_lookup(int mode, int64_t M, int64_t N, int64_t K);
void tuned_store(int mode, int64_t M, int64_t N, int64_t K, int cfg);

}  // namespace mfg
