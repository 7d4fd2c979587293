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
//      priority) is free, the oldest admitted request takes it.  A small
//      FP16 / BF16 / refined (Eq. 1, Eq. 2) request takes up to max_group
//      admitted small requests with its mode, alpha and beta into ONE
//      persistent grouped launch; any other request runs alone on the slot
//      through mfg_gemm, so large requests spread over the free slots and
//      a small request never waits for a large one's completion event.  On
//      the slot's stream each request's FP32 operands are converted into
//      stream-ordered allocations (the paper's rounding / Eq. R split / FP8
//      quantisation), then the GEMM runs; one event marks the slot's end.
// The scheduler picks the groups under the server mutex, then enqueues the
// conversions and launches (and queries completion events) with the mutex
// released, so mfg_submit / mfg_poll never wait behind HIP calls.
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
#include <cstdio>
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
#include "runtime.h"

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
    // F32 converts nothing; BF16_SPLIT6 has no preconverted form and runs
    // through mfg_gemm, whose per-stream workspace is outside the budget.
    if (m == MFG_F32 || m == MFG_BF16_SPLIT6 || r.M == 0 || r.N == 0 || r.K == 0 || r.alpha == 0.0f) {
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

// A problem the grouped kernel takes (few work items; K within its int32
// work records).  Requests that convert nothing run through mfg_gemm.
constexpr int64_t kSmallTiles = 256;
bool grouped_small(const mfg_request& r) {
    const int kind = grouped_kind(r.mode);
    if (kind < 0 || r.M * r.N >= (int64_t)512 * 512 || r.K > INT32_MAX) return false;
    if (r.M == 0 || r.N == 0 || r.K == 0 || r.alpha == 0.0f) return false;
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
    bool complete_ready(std::unique_lock<std::mutex>& lk);
    bool admit();
    bool launch_ready(std::unique_lock<std::mutex>& lk);
    void start_group(int si, const std::vector<Req*>& g);
    void enqueue_group(int si, const std::vector<Req*>& g, std::vector<int>& status, bool& event_failed);
    int run_request(Slot& sl, Req* q, bool grouped);
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

// Called with the mutex held; releases it around the event queries (the
// slots' streams and events belong to the scheduler thread alone).
bool mfg_server::complete_ready(std::unique_lock<std::mutex>& lk) {
    bool any = false;
    const int64_t t = now_ns();
    std::vector<hipError_t> ev(slots.size(), hipErrorNotReady);
    std::vector<char> query(slots.size(), 0);
    bool need_query = false;
    for (size_t i = 0; i < slots.size(); ++i) {
        const Slot& sl = slots[i];
        query[i] = sl.busy && !sl.force_ready && !dry;
        need_query |= query[i] != 0;
    }
    if (need_query) {
        lk.unlock();
        for (size_t i = 0; i < slots.size(); ++i)
            if (query[i]) ev[i] = hipEventQuery(slots[i].done);
        lk.lock();
    }
    for (size_t i = 0; i < slots.size(); ++i) {
        Slot& sl = slots[i];
        if (!sl.busy) continue;
        bool ready;
        if (sl.force_ready) {
            ready = true;
        } else if (dry) {
            ready = t >= sl.dry_end_ns;
        } else {
            const hipError_t e = ev[i];
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

// Called with the mutex held.  Picks a group for every free slot (marking
// the slot busy and its requests running), then releases the mutex while
// it enqueues their work, and records the outcome under it again.
bool mfg_server::launch_ready(std::unique_lock<std::mutex>& lk) {
    std::vector<std::pair<int, std::vector<Req*>>> picked;
    for (int si = 0; si < (int)slots.size() && !admitted.empty(); ++si) {
        if (slots[si].busy) continue;
        Req* head = admitted.front();
        std::vector<Req*> g;
        if (!grouped_small(head->r)) {
            g.push_back(head);
            admitted.pop_front();
        } else {
            const mfg_request& h = head->r;
            for (auto it = admitted.begin(); it != admitted.end() && (int)g.size() < cfg.max_group;) {
                const mfg_request& r = (*it)->r;
                if (r.mode == h.mode && r.alpha == h.alpha && r.beta == h.beta && grouped_small(r)) {
                    g.push_back(*it);
                    it = admitted.erase(it);
                } else {
                    ++it;
                }
            }
        }
        start_group(si, g);
        picked.emplace_back(si, std::move(g));
    }
    int64_t busy = 0;
    for (auto& sl : slots) busy += sl.busy ? 1 : 0;
    st.max_concurrent_slots = std::max(st.max_concurrent_slots, busy);
    if (picked.empty()) return false;
    if (dry) {
        // the dry run's executor: the fault hooks, in the order a real run meets them
        for (auto& [si, g] : picked) {
            bool grouped_failed = false;
            const bool grouped = grouped_small(g.front()->r);
            for (Req* q : g)
                if (q->footprint > 0 && fault_hit(kFaultAlloc)) q->res.status = MFG_ERR_NO_MEMORY;
            if (grouped) grouped_failed = fault_hit(kFaultLaunch);
            for (Req* q : g) {
                const mfg_request& r = q->r;
                const bool gemm = r.M > 0 && r.N > 0 && r.K > 0 && r.alpha != 0.0f;  // else no GEMM launch
                if (q->res.status == MFG_PENDING && (grouped ? grouped_failed : gemm && fault_hit(kFaultLaunch)))
                    q->res.status = MFG_ERR_HIP;
            }
            if (log_enabled())
                std::fprintf(stderr, "mfg_server: slot %d mode %d group %zu (dry run)\n", si, g.front()->r.mode,
                             g.size());
        }
        return true;
    }
    std::vector<std::vector<int>> status(picked.size());
    std::vector<char> event_failed(picked.size(), 0);
    lk.unlock();
    for (size_t i = 0; i < picked.size(); ++i) {
        bool ef = false;
        enqueue_group(picked[i].first, picked[i].second, status[i], ef);
        event_failed[i] = ef;
    }
    lk.lock();
    for (size_t i = 0; i < picked.size(); ++i) {
        const std::vector<Req*>& g = picked[i].second;
        for (size_t j = 0; j < g.size(); ++j)
            if (status[i][j] != MFG_OK && g[j]->res.status == MFG_PENDING) g[j]->res.status = status[i][j];
        if (event_failed[i]) slots[picked[i].first].force_ready = true;
    }
    return true;
}

// Convert one request's operands on the slot stream and run it, unless it
// joins the group's grouped launch (grouped: conversion only).
int mfg_server::run_request(Slot& sl, Req* q, bool grouped) {
    const mfg_request& r = q->r;
    if (q->footprint == 0)  // F32, BF16_SPLIT6, empty, K == 0 or alpha == 0: no conversion here
        return mfg_gemm(r.M, r.N, r.K, r.A, r.lda, r.B, r.ldb, r.C, r.ldc, r.alpha, r.beta, r.mode, sl.stream);
    if (fault_hit(kFaultAlloc)) return MFG_ERR_NO_MEMORY;
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
    if (s != MFG_OK || grouped) return s;
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
    return grouped_launch(kind, grouped_tile(kind), sl.d_work, two_a ? sl.d_planes : nullptr, split, g.front()->r.alpha,
                          g.front()->r.beta, sl.stream);
}

// Mutex held: the slot takes the group.
void mfg_server::start_group(int si, const std::vector<Req*>& g) {
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
    if (dry) sl.dry_end_ns = t + (int64_t)(flops / 1e5);  // 1e14 flop/s
}

// Mutex released: enqueue the group's conversions and GEMM(s) on the slot's
// stream and its completion event.  status[j] receives request j's outcome
// (MFG_OK or an error); event_failed is set when no completion event could
// be recorded (the stream has then been synchronised).
void mfg_server::enqueue_group(int si, const std::vector<Req*>& g, std::vector<int>& status, bool& event_failed) {
    Slot& sl = slots[si];
    status.assign(g.size(), MFG_OK);
    const bool grouped = grouped_small(g.front()->r);
    std::vector<Req*> small;
    std::vector<size_t> small_idx;
    for (size_t j = 0; j < g.size(); ++j) {
        status[j] = run_request(sl, g[j], grouped);
        if (status[j] == MFG_OK && grouped) {
            small.push_back(g[j]);
            small_idx.push_back(j);
        }
    }
    if (!small.empty()) {
        const int s = run_grouped(sl, small);
        if (s != MFG_OK)
            for (size_t j : small_idx) status[j] = s;
    }
    if (log_enabled())
        std::fprintf(stderr, "mfg_server: slot %d mode %d group %zu%s\n", si, g.front()->r.mode, g.size(),
                     grouped ? " grouped" : "");
    for (Req* q : g)
        if (q->ws) {
            (void)hipFreeAsync(q->ws, sl.stream);
            q->ws = nullptr;
        }
    const hipError_t e = hipEventRecord(sl.done, sl.stream);
    event_failed = false;
    if (e != hipSuccess) {
        // no event to wait for: finish the stream here and report the error
        const int code = hip_fail(e);
        (void)hipStreamSynchronize(sl.stream);
        for (size_t j = 0; j < g.size(); ++j)
            if (status[j] == MFG_OK) status[j] = code;
        event_failed = true;
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
        bool progressed = complete_ready(lk);
        progressed |= admit();
        progressed |= launch_ready(lk);
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
    fault_reload();  // MFG_FAULT as set now (also for the dry run's executor)
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
