// runtime.cpp -- error state, per-stream workspaces, device facts and the
// tuned-configuration table of libmfgemm.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>

#include "internal.h"
#include "runtime.h"

namespace mfg {

static thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    return MFG_ERR_HIP;
}

// ---------------------------------------------------------------- workspace
namespace {
struct Region {
    void* ptr = nullptr;
    size_t size = 0;
    std::mutex mu;  // held by a WsLease for the duration of one call's enqueue
};

std::mutex g_map_mu;
// Regions are never erased, so references stay valid; released at exit by
// the process teardown (freeing after the HIP runtime is gone is unsafe).
std::map<std::tuple<int, int, hipStream_t>, Region*> g_regions;

Region* region_for(int slot, hipStream_t s, int* dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (dev_out) *dev_out = dev;
    std::lock_guard<std::mutex> g(g_map_mu);
    auto key = std::make_tuple(slot, dev, s);
    auto it = g_regions.find(key);
    if (it != g_regions.end()) return it->second;
    Region* r = new Region();
    g_regions.emplace(key, r);
    return r;
}

void* grow(Region* r, hipStream_t s, size_t bytes, int* status) {
    if (r->size >= bytes && r->ptr != nullptr) return r->ptr;
    if (r->ptr != nullptr) {
        // Work already enqueued on this stream may still read the old region.
        if (hipStreamSynchronize(s) != hipSuccess || hipFree(r->ptr) != hipSuccess) {
            *status = MFG_ERR_HIP;
            r->ptr = nullptr;
            r->size = 0;
            return nullptr;
        }
        r->ptr = nullptr;
        r->size = 0;
    }
    if (fault_hit(kFaultAlloc)) {
        *status = MFG_ERR_NO_MEMORY;
        return nullptr;
    }
    size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    want = (want + ((size_t)2 << 20) - 1) / ((size_t)2 << 20) * ((size_t)2 << 20);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *status = MFG_ERR_NO_MEMORY;
        return nullptr;
    }
    r->ptr = p;
    r->size = want;
    return p;
}
}  // namespace

WsLease::WsLease(hipStream_t s, size_t bytes) {
    Region* r = region_for(0, s, nullptr);
    lock_ = std::unique_lock<std::mutex>(r->mu);
    ptr_ = grow(r, s, bytes, &status_);
}

void* workspace(hipStream_t s, size_t bytes, int* status) {
    Region* r = region_for(0, s, nullptr);
    return grow(r, s, bytes, status);
}

void* partials_ws(hipStream_t s, size_t bytes, int* status) {
    Region* r = region_for(1, s, nullptr);
    std::lock_guard<std::mutex> g(r->mu);
    return grow(r, s, bytes, status);
}

int device_cu_count() {
    static std::mutex mu;
    static std::map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev] = n;
    return n;
}

// ---------------------------------------------------------- fault injection
namespace {
std::atomic<int64_t> g_fault_left[kFaultKinds];  // calls until the injected fault; <= 0: off
std::once_flag g_fault_env_once;

int64_t parse_fault(const char* spec, const char* key) {
    if (!spec) return 0;
    const char* p = std::strstr(spec, key);
    if (!p) return 0;
    p += std::strlen(key);
    if (*p != ':') return 0;
    const long long n = std::strtoll(p + 1, nullptr, 10);
    return n > 0 ? (int64_t)n : 0;
}
}  // namespace

void fault_arm(int64_t launch_n, int64_t alloc_n) {
    g_fault_left[kFaultLaunch].store(launch_n > 0 ? launch_n : 0);
    g_fault_left[kFaultAlloc].store(alloc_n > 0 ? alloc_n : 0);
}

void fault_reload() {
    const char* spec = std::getenv("MFG_FAULT");
    fault_arm(parse_fault(spec, "launch"), parse_fault(spec, "alloc"));
}

bool fault_hit(int kind) {
    std::call_once(g_fault_env_once, fault_reload);
    if (g_fault_left[kind].load(std::memory_order_relaxed) <= 0) return false;
    return g_fault_left[kind].fetch_sub(1) == 1;
}

bool log_enabled() {
    static const bool on = [] {
        const char* p = std::getenv("MFG_LOG");
        return p && *p && *p != '0';
    }();
    return on;
}

// ------------------------------------------------------------- tuned table
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;
bool g_tune_env_loaded = false;
}  // namespace

int size_bucket(int64_t x) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << (b + 1)) <= x) ++b;
    return b;
}

static void load_env_table_locked();

int tuned_lookup(int mode, int64_t M, int64_t N, int64_t K) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_env_table_locked();
    auto it = g_tune.find(std::make_tuple(mode, size_bucket(M), size_bucket(N), size_bucket(K)));
    return it == g_tune.end() ? -1 : it->second;
}

void tuned_store(int mode, int64_t M, int64_t N, int64_t K, int cfg) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[std::make_tuple(mode, size_bucket(M), size_bucket(N), size_bucket(K))] = cfg;
}

static int load_table_locked(const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return MFG_ERR_INVALID_ARG;
    int mode, mb, nb, kb, cfg;
    int rc = MFG_OK;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        const int got = std::sscanf(line, "%d %d %d %d %d", &mode, &mb, &nb, &kb, &cfg);
        const bool mode_ok = got == 5 && ((mode >= 0 && mode < MFG_NUM_MODES) ||
                                          (mode >= kGroupedTuneBase && mode < kGroupedTuneBase + MFG_NUM_MODES));
        if (!mode_ok || cfg < 0) {
            rc = MFG_ERR_INVALID_ARG;
            continue;
        }
        g_tune[std::make_tuple(mode, mb, nb, kb)] = cfg;
    }
    std::fclose(f);
    return rc;
}

static void load_env_table_locked() {
    if (g_tune_env_loaded) return;
    g_tune_env_loaded = true;
    const char* p = std::getenv("MFG_TUNE_TABLE");
    if (p && *p) (void)load_table_locked(p);
}

}  // namespace mfg

extern "C" int mfg_last_hip_error(void) { return mfg::g_last_hip_error; }

extern "C" int mfg_tune_save(const char* path) {
    if (!path) return MFG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(mfg::g_tune_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return MFG_ERR_INVALID_ARG;
    std::fprintf(f, "# mode mbucket nbucket kbucket config  (bucket = floor(log2(size)))\n");
    for (const auto& kv : mfg::g_tune)
        std::fprintf(f, "%d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                     std::get<3>(kv.first), kv.second);
    std::fclose(f);
    return MFG_OK;
}

extern "C" int mfg_tune_load(const char* path) {
    if (!path) return MFG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(mfg::g_tune_mu);
    return mfg::load_table_locked(path);
}

extern "C" int mfg_tune_clear(void) {
    std::lock_guard<std::mutex> g(mfg::g_tune_mu);
    mfg::g_tune.clear();
    mfg::g_tune_env_loaded = true;
    return MFG_OK;
}

extern "C" int mfg_fault_inject(int64_t launch_n, int64_t alloc_n) {
    if (launch_n < 0 || alloc_n < 0) return MFG_ERR_INVALID_ARG;
    mfg::fault_hit(mfg::kFaultLaunch);  // reads MFG_FAULT once, so it cannot override this call later
    mfg::fault_arm(launch_n, alloc_n);
    return MFG_OK;
}
