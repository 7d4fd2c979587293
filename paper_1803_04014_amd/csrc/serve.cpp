// serve.cpp -- the request loop of libmfgemm (mfg_server_*): continuous
// batching of GEMM requests of mixed sizes and modes with admission by an HBM
// budget.
//
// One scheduler thread per server owns every HIP call of the server.  Its
// loop, after each wake-up (a submission, a completion, a short poll tick):
//   1. completions: a slot whose completion event has fired releases its
//      requests (timestamps, status) and their converted-operand footprint;
//   2. admission, first come first served: the oldest waiting request is
//      admitted while  bytes_in_use + footprint <= hbm_budget_bytes;  a request
//      that does not fit blocks the ones behind it (no starvation of large
//      requests);
//   3. launches: while a slot (one non-blocking HIP stream of default
//      priority) is free, the oldest admitted request picks a group of up to
//      max_group admitted requests with its mode (and its alpha and beta,
//      which a grouped launch shares).  On the slot's stream
//      each request's FP32 operands are converted into stream-ordered
//      allocations (the paper's rounding / Eq. R split / FP8 quantisation),
//      then the GEMMs run: small FP16 / BF16 / refined (Eq. 1, Eq. 2)
//      problems of the group as ONE persistent grouped launch, every other
//      problem through mfg_gemm on
//      the converted operands; one event marks the group's end.
// Every kernel the server runs is one that mfg_gemm / the grouped plan would
// run for the same problem, and all 16-bit kernels share one accumulation
// order, so a request's result does not depend on what it was batched with.
//
// device = -1 is a dry run for testing the scheduler: it validates, admits,
// groups and accounts exactly as above but makes no HIP call, never touches
// A, B or C, and completes a group after flops / 1e14 seconds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "mfgemm.h"

namespace mfg {
namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}
int64_t up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

enum State { QUEUED, ADMITTED, RUNNING, DONE };

struct Req {
    uint64_t ticket = 0;
    mfg_request r{};
    mfg_result res{};
    int64_t footprint = 0;  // bytes of converted operands
    int64_t lda_c = 0, ldb_c = 0, off_b = 0;
    void* ws = nullptr;
    State state = QUEUED;
};

// Leading dimensions of the converted operands and the workspace size.
void plan_footprint(Req& q) {
    const mfg_request& r = q.r;
    const int m = r.mode;
    if (m == MFG_F32 || r.M == 0 || r.N == 0 || r.K == 0 || r.alpha == 0.0f) {
        q.footprint = 0;
        return;
    }
    const int64_t al = (m == MFG_FP8_E4M3) ? 16 : 8;
    q.lda_c = up(r.K, al);
    q.ldb_c = up(r.N, al);
    const int mb = (m == MFG_F16_REFINE_A) ? MFG_F16 : m;  // B keeps only its head under Eq. 1
    const int64_t ba = mfg_convert_bytes(r.M, r.K, q.lda_c, m);
    const int64_t bb = mfg_convert_bytes(r.K, r.N, q.ldb_c, mb);
    q.off_b = up(ba, 256);
    q.footprint = q.off_b + up(bb, 256);
}

// The grouped kernel's kind for a request mode (-1: not a grouped mode).
int grouped_kind(int mode) {
    switch (mode) {
        case MFG_F16: return K_F16;
        case MFG_BF16: return K_BF16;
        case MFG_F16_REFINE_A: return K_REFINE_A;
        case MFG_F16_SPLIT3: return K_SPLIT3;
        case MFG_F16_SPLIT4: return K_SPLIT4;
        case MFG_BF16_SPLIT3: return K_BF16_SPLIT3;
        default: return -1;
    }
}

// A problem the grouped kernel takes (few work items).
constexpr int64_t kSmallTiles = 256;
bool grouped_small(const mfg_request& r) {
    const int kind = grouped_kind(r.mode);
    if (kind < 0 || r.M * r.N >= (int64_t)512 * 512) return false;
    const int t = grouped_tile(kind);
    return cdiv(r.M, t) * cdiv(r.N, t) <= kSmallTiles;
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    bool force_ready = false;  // the group's end is already known (its event could not be recorded)
    int64_t dry_end_ns = 0;
    std::vector<Req*> running;
    std::vector<GroupedDesc> h_desc;  // the group's problems (host side)
    GroupedWork* h_work = nullptr;
    GroupedWork* d_work = nullptr;
    int64_t* h_planes = nullptr;  // refined modes: residual-plane offsets, two per work item
    int64_t* d_planes = nullptr;
};

}  // namespace
}  // namespace mfg

using namespace mfg;

struct mfg_server {
    mfg_server_config cfg{};
    bool dry = false;
    std::mutex mu;
    std::condition_variable cv;       // scheduler wake-ups
    std::condition_variable cv_done;  // completions (drain)
    std::thread thr;
    bool stop = false;
    int init_status = MFG_PENDING;
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::deque<Req*> queued, admitted;
    std::vector<Slot> slots;
    int64_t unfinished = 0;
    mfg_server_stats st{};
    int64_t work_cap = 0;

    int init_device();
    void release_device();
    void loop();
    bool complete_ready();
    bool admit();
    bool launch_ready();
    void launch_group(int si, std::vector<Req*>& g);
    int run_request(Slot& sl, Req* q, bool& grouped);
    int run_grouped(Slot& sl, const std::vector<Req*>& g);
};

int mfg_server::init_device() {
    MFG_HIP_CHECK(hipSetDevice(cfg.device));
    int pools = 0;  // converted operands live in stream-ordered allocations
    MFG_HIP_CHECK(hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, cfg.device));
    if (!pools) return MFG_ERR_UNSUPPORTED;
    work_cap = (int64_t)cfg.max_group * kSmallTiles;
    for (auto& sl : slots) {
        MFG_HIP_CHECK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
        MFG_HIP_CHECK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        sl.h_desc.resize((size_t)cfg.max_group);
        MFG_HIP_CHECK(hipHostMalloc((void**)&sl.h_work, sizeof(GroupedWork) * work_cap, 0));
        MFG_HIP_CHECK(hipMalloc((void**)&sl.d_work, sizeof(GroupedWork) * work_cap));
        MFG_HIP_CHECK(hipHostMalloc((void**)&sl.h_planes, sizeof(int64_t) * 2 * work_cap, 0));
        MFG_HIP_CHECK(hipMalloc((void**)&sl.d_planes, sizeof(int64_t) * 2 * work_cap));
    }
    return MFG_OK;
}

void mfg_server::release_device() {
    for (auto& sl : slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_work) (void)hipHostFree(sl.h_work);
        if (sl.d_work) (void)hipFree(sl.d_work);
        if (sl.h_planes) (void)hipHostFree(sl.h_planes);
        if (sl.d_planes) (void)hipFree(sl.d_planes);
        sl = Slot{};
    }
}

bool mfg_server::complete_ready() {
    bool any = false;
    const int64_t t = now_ns();
    for (auto& sl : slots) {
        if (!sl.busy) continue;
        bool ready;
        if (sl.force_ready) {
            ready = true;
        } else if (dry) {
            ready = t >= sl.dry_end_ns;
        } else {
            const hipError_t e = hipEventQuery(sl.done);
            ready = e != hipErrorNotReady;
            if (ready && e != hipSuccess) {
                const int code = hip_fail(e);
                for (Req* q : sl.running)
                    if (q->res.status == MFG_PENDING) q->res.status = code;
            }
        }
        if (!ready) continue;
        const int64_t t_end = now_ns();
        for (Req* q : sl.running) {
            q->res.t_end_ns = t_end;
            if (q->res.status == MFG_PENDING) q->res.status = MFG_OK;
            if (q->res.status == MFG_OK) ++st.completed;
            else ++st.failed;
            q->state = DONE;
            st.bytes_in_use -= (uint64_t)q->footprint;
            --unfinished;
        }
        sl.running.clear();
        sl.busy = false;
        sl.force_ready = false;
        any = true;
    }
    if (any) cv_done.notify_all();
    return any;
}

bool mfg_server::admit() {
    bool any = false;
    while (!queued.empty()) {
        Req* q = queued.front();
        if (st.bytes_in_use + (uint64_t)q->footprint > cfg.hbm_budget_bytes) break;
        queued.pop_front();
        st.bytes_in_use += (uint64_t)q->footprint;
        st.peak_bytes_in_use = std::max(st.peak_bytes_in_use, st.bytes_in_use);
        q->state = ADMITTED;
        q->res.t_admit_ns = now_ns();
        admitted.push_back(q);
        any = true;
    }
    return any;
}

bool mfg_server::launch_ready() {
    bool any = false;
    for (int si = 0; si < (int)slots.size() && !admitted.empty(); ++si) {
        if (slots[si].busy) continue;
        const mfg_request& h = admitted.front()->r;
        const int mode = h.mode;
        const float al = h.alpha, be = h.beta;
        std::vector<Req*> g;
        for (auto it = admitted.begin(); it != admitted.end() && (int)g.size() < cfg.max_group;) {
            const mfg_request& r = (*it)->r;
            if (r.mode == mode && r.alpha == al && r.beta == be) {
                g.push_back(*it);
                it = admitted.erase(it);
            } else {
                ++it;
            }
        }
        launch_group(si, g);
        any = true;
    }
    int64_t busy = 0;
    for (auto& sl : slots) busy += sl.busy ? 1 : 0;
    st.max_concurrent_slots = std::max(st.max_concurrent_slots, busy);
    return any;
}

// Convert one request's operands on the slot stream; run it unless it joins
// the group's grouped launch.
int mfg_server::run_request(Slot& sl, Req* q, bool& grouped) {
    const mfg_request& r = q->r;
    grouped = false;
    if (q->footprint == 0)  // F32, empty, K == 0 or alpha == 0: no conversion
        return mfg_gemm(r.M, r.N, r.K, r.A, r.lda, r.B, r.ldb, r.C, r.ldc, r.alpha, r.beta, r.mode, sl.stream);
    hipError_t e = hipMallocAsync(&q->ws, (size_t)q->footprint, sl.stream);
    if (e != hipSuccess) {
        q->ws = nullptr;
        (void)hipGetLastError();
        return MFG_ERR_NO_MEMORY;
    }
    char* wa = static_cast<char*>(q->ws);
    char* wb = wa + q->off_b;
    const int mb = (r.mode == MFG_F16_REFINE_A) ? MFG_F16 : r.mode;
    int s = mfg_convert(r.M, r.K, r.A, r.lda, wa, q->lda_c, r.mode, sl.stream);
    if (s == MFG_OK) s = mfg_convert(r.K, r.N, r.B, r.ldb, wb, q->ldb_c, mb, sl.stream);
    if (s != MFG_OK) return s;
    if (grouped_small(r)) {
        grouped = true;
        return MFG_OK;
    }
    return mfg_gemm(r.M, r.N, r.K, wa, q->lda_c, wb, q->ldb_c, r.C, r.ldc, r.alpha, r.beta,
                    r.mode | MFG_IN_PRECONVERTED, sl.stream);
}

// One persistent grouped launch over the group's small problems (one mode;
// the same descriptors and work order as a grouped plan; one alpha, beta).
int mfg_server::run_grouped(Slot& sl, const std::vector<Req*>& g) {
    const int mode = g.front()->r.mode, kind = grouped_kind(mode);
    // converted refined operands: head plane, then residual plane (B: only
    // for the two-sided splits; Eq. 1 keeps B's head alone)
    const bool two_a = kind >= K_REFINE_A, two_b = kind >= K_SPLIT3;
    int64_t nd = 0;
    for (Req* q : g) {
        const mfg_request& r = q->r;
        GroupedDesc& d = sl.h_desc[nd++];
        d.M = r.M, d.N = r.N, d.K = r.K, d.lda = q->lda_c, d.ldb = q->ldb_c, d.ldc = r.ldc;
        d.A = static_cast<const uint16_t*>(q->ws);
        d.B = reinterpret_cast<const uint16_t*>(static_cast<const char*>(q->ws) + q->off_b);
        d.C = r.C;
        d.vec = 1;  // workspace planes: 256-byte aligned, ld a multiple of 8
        d.pad = 0;
        d.pa = two_a ? r.M * q->lda_c : 0;
        d.pb = two_b ? r.K * q->ldb_c : 0;
    }
    GroupedSplit split{};
    std::vector<GroupedWork> work;
    std::vector<int64_t> planes;
    build_grouped_work(sl.h_desc.data(), nd, work, split, two_a ? &planes : nullptr, grouped_tile(kind));
    const int64_t nw = (int64_t)work.size();  // <= max_group * kSmallTiles (grouped_small)
    if (nw > work_cap) return MFG_ERR_INTERNAL;
    std::copy(work.begin(), work.end(), sl.h_work);
    MFG_HIP_CHECK(hipMemcpyAsync(sl.d_work, sl.h_work, sizeof(GroupedWork) * nw, hipMemcpyHostToDevice, sl.stream));
    if (two_a) {
        std::copy(planes.begin(), planes.end(), sl.h_planes);
        MFG_HIP_CHECK(hipMemcpyAsync(sl.d_planes, sl.h_planes, sizeof(int64_t) * 2 * nw, hipMemcpyHostToDevice,
                                     sl.stream));
    }
    return grouped_launch(kind, sl.d_work, two_a ? sl.d_planes : nullptr, split, g.front()->r.alpha,
                          g.front()->r.beta, sl.stream);
}

void mfg_server::launch_group(int si, std::vector<Req*>& g) {
    Slot& sl = slots[si];
    const int64_t t = now_ns();
    double flops = 0.0;
    for (Req* q : g) {
        q->state = RUNNING;
        q->res.t_start_ns = t;
        q->res.slot = si;
        q->res.group_size = (int64_t)g.size();
        flops += q->res.flops;
    }
    sl.running = g;
    sl.busy = true;
    ++st.launches;
    if (dry) {
        sl.dry_end_ns = t + (int64_t)(flops / 1e5);  // 1e14 flop/s
        return;
    }
    std::vector<Req*> small;
    for (Req* q : g) {
        bool grouped = false;
        const int s = run_request(sl, q, grouped);
        if (s != MFG_OK) q->res.status = s;
        else if (grouped) small.push_back(q);
    }
    if (!small.empty()) {
        const int s = run_grouped(sl, small);
        if (s != MFG_OK)
            for (Req* q : small) q->res.status = s;
    }
    for (Req* q : g)
        if (q->ws) {
            (void)hipFreeAsync(q->ws, sl.stream);
            q->ws = nullptr;
        }
    const hipError_t e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) {
        // no event to wait for: finish the stream here and report the error
        const int code = hip_fail(e);
        (void)hipStreamSynchronize(sl.stream);
        for (Req* q : g)
            if (q->res.status == MFG_PENDING) q->res.status = code;
        sl.force_ready = true;
    }
}

void mfg_server::loop() {
    std::unique_lock<std::mutex> lk(mu);
    if (!dry) {
        init_status = init_device();
        if (init_status != MFG_OK) {
            cv_done.notify_all();
            return;
        }
    }
    init_status = MFG_OK;
    cv_done.notify_all();
    while (true) {
        bool progressed = complete_ready();
        progressed |= admit();
        progressed |= launch_ready();
        if (progressed) continue;
        bool busy = false;
        for (auto& sl : slots) busy |= sl.busy;
        if (stop && !busy && queued.empty() && admitted.empty()) break;
        if (busy) cv.wait_for(lk, std::chrono::microseconds(20));
        else cv.wait(lk);
    }
}

// ------------------------------------------------------------------ C ABI
extern "C" int mfg_server_create(const mfg_server_config* cfg, mfg_server** out) {
    if (!cfg || !out) return MFG_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > 64 || cfg->max_group < 1 || cfg->max_group > 4096 || cfg->device < -1 ||
        cfg->reserved != 0)
        return MFG_ERR_INVALID_ARG;
    try {
        std::unique_ptr<mfg_server> s(new mfg_server());
        s->cfg = *cfg;
        s->dry = cfg->device == -1;
        s->slots.resize((size_t)cfg->slots);
        s->thr = std::thread([p = s.get()] { p->loop(); });
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_done.wait(lk, [&] { return s->init_status != MFG_PENDING; });
        }
        if (s->init_status != MFG_OK) {
            const int code = s->init_status;
            s->thr.join();
            if (!s->dry) s->release_device();
            return code;
        }
        *out = s.release();
        return MFG_OK;
    } catch (const std::bad_alloc&) {
        return MFG_ERR_NO_MEMORY;
    } catch (...) {
        return MFG_ERR_INTERNAL;
    }
}

extern "C" int mfg_submit(mfg_server* s, const mfg_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return MFG_ERR_INVALID_ARG;
    const int m = req->mode;
    if (m < 0 || m >= MFG_NUM_MODES || req->reserved != 0) return MFG_ERR_INVALID_ARG;
    int v = mfg_validate_gemm(req->M, req->N, req->K, req->A, req->lda, req->B, req->ldb, req->C, req->ldc, m);
    if (v != MFG_OK) return v;
    try {
        std::unique_ptr<Req> q(new Req());
        q->r = *req;
        plan_footprint(*q);
        if ((uint64_t)q->footprint > s->cfg.hbm_budget_bytes) return MFG_ERR_OVER_BUDGET;
        q->res.status = MFG_PENDING;
        q->res.slot = -1;
        q->res.flops = 2.0 * (double)req->M * (double)req->N * (double)req->K;
        q->res.t_submit_ns = now_ns();
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return MFG_ERR_INVALID_ARG;
        q->ticket = s->next_ticket++;
        *ticket = q->ticket;
        Req* raw = q.get();
        s->reqs.emplace(raw->ticket, std::move(q));
        s->queued.push_back(raw);
        ++s->unfinished;
        ++s->st.submitted;
        s->cv.notify_one();
        return MFG_OK;
    } catch (const std::bad_alloc&) {
        return MFG_ERR_NO_MEMORY;
    } catch (...) {
        return MFG_ERR_INTERNAL;
    }
}

extern "C" int mfg_poll(mfg_server* s, uint64_t ticket, mfg_result* out) {
    if (!s) return MFG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return MFG_ERR_UNKNOWN_TICKET;
    Req* q = it->second.get();
    if (out) *out = q->res;
    if (q->state != DONE) {
        if (out) out->status = MFG_PENDING;
        return MFG_PENDING;
    }
    const int status = q->res.status;
    s->reqs.erase(it);
    return status;
}

extern "C" int mfg_server_drain(mfg_server* s) {
    if (!s) return MFG_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.notify_one();
    s->cv_done.wait(lk, [&] { return s->unfinished == 0; });
    return MFG_OK;
}

extern "C" int mfg_server_get_stats(mfg_server* s, mfg_server_stats* out) {
    if (!s || !out) return MFG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return MFG_OK;
}

extern "C" int mfg_server_destroy(mfg_server* s) {
    if (!s) return MFG_ERR_INVALID_ARG;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->unfinished == 0; });
        s->stop = true;
        s->cv.notify_one();
    }
    s->thr.join();
    if (!s->dry) s->release_device();
    delete s;
    return MFG_OK;
}
