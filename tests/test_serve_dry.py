"""The serving loop's scheduler on the CPU (mfg_server with device = -1: a dry
run that validates, admits, groups and accounts but computes nothing).

Checks the admission invariant (bytes in use never above the budget), first-
come-first-served admission, grouping by mode, ticket life cycle, footprints
and argument errors.  No GPU: the dry run makes no HIP call and never
dereferences A, B or C, so fake device addresses stand in for buffers.
"""
import threading
import time

import numpy as np
import pytest

import paper_1803_04014_amd as mfg
import workloads
from paper_1803_04014_amd import capi

FAKE_A, FAKE_B, FAKE_C = 0x7F0000000000, 0x7F1000000000, 0x7F2000000000


def up(x, m):
    return -(-x // m) * m


def footprint(M, N, K, mode):
    """Converted-operand bytes of one request, from the header's definition."""
    if mode == "f32" or M == 0 or N == 0 or K == 0:
        return 0
    al = 16 if mode == "fp8" else 8
    lda, ldb = up(K, al), up(N, al)
    if mode == "fp8":  # codes, then the tile scales at an aligned offset (mfg_convert_bytes)
        ba = mfg.lib().mfg_convert_bytes(M, K, lda, mfg.mode_of("fp8"))
        bb = mfg.lib().mfg_convert_bytes(K, N, ldb, mfg.mode_of("fp8"))
    else:
        planes_a = 2 if mode in ("refine_a", "split3", "split4") else 1
        planes_b = 2 if mode in ("split3", "split4") else 1
        ba, bb = planes_a * M * lda * 2, planes_b * K * ldb * 2
    return up(ba, 256) + up(bb, 256)


def submit(s, M, N, K, mode, alpha=1.0, beta=0.0):
    return s.submit(None, None, None, mode, alpha, beta, M=M, N=N, K=K, A_ptr=FAKE_A, B_ptr=FAKE_B,
                    C_ptr=FAKE_C, lda=max(K, 1), ldb=max(N, 1), ldc=max(N, 1))


def wait_all(s, tickets, timeout=60.0):
    out, t0 = {}, time.time()
    pending = list(tickets)
    while pending:
        nxt = []
        for t in pending:
            st, r = s.poll(t)
            if st == capi.MFG_PENDING:
                nxt.append(t)
            else:
                r["status"] = st
                out[t] = r
        pending = nxt
        assert time.time() - t0 < timeout, "requests did not finish"
        if pending:
            time.sleep(0.001)
    return out


def test_footprints_match_definition():
    for mode in ("f16", "bf16", "refine_a", "split3", "split4", "fp8", "f32"):
        for (M, N, K) in ((100, 37, 250), (1, 1, 1), (128, 128, 128), (300, 17, 9)):
            s = mfg.Server(1 << 40, slots=1, device=-1, max_group=1)
            t = submit(s, M, N, K, mode)
            wait_all(s, [t])
            assert s.stats()["peak_bytes_in_use"] == footprint(M, N, K, mode), (mode, M, N, K)
            assert s.stats()["bytes_in_use"] == 0
            s.close()


def test_admission_never_exceeds_budget_and_all_complete():
    budget = 48 << 20
    s = mfg.Server(budget, slots=4, device=-1, max_group=8)
    trace = workloads.serving_trace(7, 1000.0, 300, lo=32, hi=2048)
    tickets = []
    for r in trace:
        try:
            tickets.append((submit(s, r["M"], r["N"], r["K"], r["mode"]), r))
        except mfg.MfgError as e:
            assert e.status == capi.MFG_ERR_OVER_BUDGET
            assert footprint(r["M"], r["N"], r["K"], r["mode"]) > budget
    res = wait_all(s, [t for t, _ in tickets])
    st = s.stats()
    assert st["peak_bytes_in_use"] <= budget
    assert st["bytes_in_use"] == 0
    assert st["completed"] == len(tickets) and st["failed"] == 0
    assert 1 <= st["max_concurrent_slots"] <= 4
    for t, r in tickets:
        x = res[t]
        assert x["status"] == 0
        assert x["t_submit_ns"] <= x["t_admit_ns"] <= x["t_start_ns"] <= x["t_end_ns"]
        assert 1 <= x["group_size"] <= 8 and 0 <= x["slot"] < 4
        assert x["flops"] == 2.0 * r["M"] * r["N"] * r["K"]
    s.close()


def test_admission_is_first_come_first_served():
    # each request alone nearly fills the budget: admissions happen one at a time, in order
    M = N = K = 1024
    fp = footprint(M, N, K, "f16")
    s = mfg.Server(fp + fp // 2, slots=2, device=-1, max_group=4)
    tickets = [submit(s, M, N, K, "f16") for _ in range(12)]
    res = wait_all(s, tickets)
    admits = [res[t]["t_admit_ns"] for t in tickets]
    assert admits == sorted(admits)
    assert s.stats()["peak_bytes_in_use"] == fp
    assert all(res[t]["group_size"] == 1 for t in tickets)
    s.close()


def test_requests_of_one_mode_are_grouped():
    # one slot kept busy by a large request; the small ones that wait behind it
    # leave in groups of at most max_group, one mode per group
    s = mfg.Server(1 << 40, slots=1, device=-1, max_group=5)
    big = submit(s, 8192, 8192, 8192, "f16")  # 11 ms of dry-run time
    small = [(submit(s, 64, 64, 64, m), m) for m in ["bf16", "split3"] * 6]
    res = wait_all(s, [big] + [t for t, _ in small])
    groups = {}
    for t, m in small:
        key = (res[t]["t_start_ns"], res[t]["slot"])
        groups.setdefault(key, set()).add(m)
        assert res[t]["t_start_ns"] >= res[big]["t_end_ns"] or res[t]["slot"] != res[big]["slot"]
    assert all(len(ms) == 1 for ms in groups.values())
    sizes = sorted(res[t]["group_size"] for t, _ in small)
    assert max(sizes) == 5
    assert s.stats()["launches"] < 1 + len(small)
    s.close()


def test_alpha_beta_split_groups():
    s = mfg.Server(1 << 40, slots=1, device=-1, max_group=16)
    big = submit(s, 8192, 8192, 8192, "f16", 3.0, 0.0)  # groups with neither set
    a = [submit(s, 32, 32, 32, "f16", 1.0, 0.0) for _ in range(3)]
    b = [submit(s, 32, 32, 32, "f16", 2.0, 1.0) for _ in range(3)]
    res = wait_all(s, [big] + a + b)
    assert len({res[t]["t_start_ns"] for t in a}) == 1 and len({res[t]["t_start_ns"] for t in b}) == 1
    assert res[a[0]]["t_start_ns"] != res[b[0]]["t_start_ns"]
    s.close()


def test_ticket_life_cycle():
    s = mfg.Server(1 << 30, slots=2, device=-1, max_group=4)
    t = submit(s, 16, 16, 16, "f16")
    res = wait_all(s, [t])
    assert res[t]["status"] == 0
    st, _ = s.poll(t)  # released by the final poll
    assert st == capi.MFG_ERR_UNKNOWN_TICKET
    st, _ = s.poll(123456789)
    assert st == capi.MFG_ERR_UNKNOWN_TICKET
    s.close()


def test_empty_and_zero_k_requests_complete():
    s = mfg.Server(1 << 20, slots=1, device=-1, max_group=4)
    ts = [submit(s, 0, 8, 8, "split3"), submit(s, 8, 0, 8, "f16"), submit(s, 8, 8, 0, "fp8")]
    res = wait_all(s, ts)
    assert all(res[t]["status"] == 0 for t in ts)
    assert s.stats()["peak_bytes_in_use"] == 0
    s.close()


def test_over_budget_and_invalid_requests():
    s = mfg.Server(1 << 20, slots=1, device=-1, max_group=4)
    with pytest.raises(mfg.MfgError) as e:
        submit(s, 1024, 1024, 1024, "f16")  # 4 MiB of converted operands
    assert e.value.status == capi.MFG_ERR_OVER_BUDGET
    for bad in (dict(M=-1, N=8, K=8), dict(M=8, N=8, K=8, lda=4)):
        with pytest.raises(mfg.MfgError) as e:
            s.submit(None, None, None, "f16", M=bad["M"], N=bad["N"], K=bad["K"], A_ptr=FAKE_A, B_ptr=FAKE_B,
                     C_ptr=FAKE_C, lda=bad.get("lda", 8), ldb=8, ldc=8)
        assert e.value.status == capi.MFG_ERR_INVALID_ARG
    req = capi.mfg_request(8, 8, 8, 8, 8, 8, FAKE_A, FAKE_B, FAKE_C, 1.0, 0.0, 1 | capi.MFG_IN_PRECONVERTED, 0)
    t = __import__("ctypes").c_uint64()
    assert mfg.lib().mfg_submit(s.handle, req, t) == capi.MFG_ERR_INVALID_ARG
    req = capi.mfg_request(8, 8, 8, 8, 8, 8, FAKE_A, FAKE_B, FAKE_C, 1.0, 0.0, 1, 7)
    assert mfg.lib().mfg_submit(s.handle, req, t) == capi.MFG_ERR_INVALID_ARG
    req = capi.mfg_request(8, 8, 8, 8, 8, 8, None, FAKE_B, FAKE_C, 1.0, 0.0, 1, 0)
    assert mfg.lib().mfg_submit(s.handle, req, t) == capi.MFG_ERR_INVALID_ARG
    assert s.stats()["submitted"] == 0
    s.close()


@pytest.mark.parametrize("cfg", [(0, 4), (65, 4), (1, 0), (1, 5000)])
def test_invalid_server_config(cfg):
    slots, max_group = cfg
    with pytest.raises(mfg.MfgError) as e:
        mfg.Server(1 << 20, slots=slots, device=-1, max_group=max_group)
    assert e.value.status == capi.MFG_ERR_INVALID_ARG


def test_concurrent_submitters_and_drain():
    budget = 16 << 20
    s = mfg.Server(budget, slots=3, device=-1, max_group=6)
    tickets, lock = [], threading.Lock()

    def worker(seed):
        g = np.random.default_rng(seed)
        for _ in range(60):
            M, N, K = (int(x) for x in g.integers(16, 700, size=3))
            mode = ["f16", "bf16", "split3", "fp8", "f32"][int(g.integers(0, 5))]
            t = submit(s, M, N, K, mode)
            with lock:
                tickets.append(t)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    s.drain()
    st = s.stats()
    assert st["submitted"] == st["completed"] == 240 and st["failed"] == 0
    assert st["peak_bytes_in_use"] <= budget and st["bytes_in_use"] == 0
    assert len(set(tickets)) == 240
    res = wait_all(s, tickets)
    assert all(r["status"] == 0 for r in res.values())
    s.close()


def _arm(launch_n=0, alloc_n=0):
    assert mfg.lib().mfg_fault_inject(launch_n, alloc_n) == 0


def test_injected_launch_fault_fails_one_request_and_serving_continues():
    s = mfg.Server(1 << 40, slots=1, device=-1, max_group=1)
    _arm(launch_n=3)
    try:
        # 1024^3: not a grouped size, so one launch per request, in submission order
        tickets = [submit(s, 1024, 1024, 1024, "f16") for _ in range(6)]
        res = wait_all(s, tickets)
    finally:
        _arm()
    status = [res[t]["status"] for t in tickets]
    assert status == [0, 0, capi.MFG_ERR_HIP, 0, 0, 0]
    st = s.stats()
    assert st["failed"] == 1 and st["completed"] == 5 and st["bytes_in_use"] == 0
    # the server keeps serving after the failure
    t = submit(s, 64, 64, 64, "split3")
    assert wait_all(s, [t])[t]["status"] == 0
    s.close()


def test_injected_alloc_fault_marks_request_out_of_memory():
    s = mfg.Server(1 << 40, slots=2, device=-1, max_group=1)
    _arm(alloc_n=2)
    try:
        tickets = []
        for _ in range(5):  # one at a time, so allocations happen in submission order
            tickets.append(submit(s, 1024, 1024, 1024, "split3"))
            s.drain()
        res = wait_all(s, tickets)
    finally:
        _arm()
    assert [res[t]["status"] for t in tickets] == [0, capi.MFG_ERR_NO_MEMORY, 0, 0, 0]
    assert s.stats()["failed"] == 1 and s.stats()["bytes_in_use"] == 0
    s.close()


def test_injected_fault_in_grouped_launch_fails_its_group_only():
    s = mfg.Server(1 << 40, slots=1, device=-1, max_group=4)
    big = submit(s, 8192, 8192, 8192, "f16")  # holds the one slot while the small ones queue
    small = [submit(s, 48, 48, 48, "bf16") for _ in range(8)]
    _arm(launch_n=2)  # the first group after the big request
    try:
        res = wait_all(s, [big] + small)
    finally:
        _arm()
    assert res[big]["status"] == 0
    failed = [t for t in small if res[t]["status"] != 0]
    assert len(failed) == 4 and all(res[t]["status"] == capi.MFG_ERR_HIP for t in failed)
    assert len({res[t]["t_start_ns"] for t in failed}) == 1  # one grouped launch
    assert s.stats()["failed"] == 4
    s.close()


def test_fault_from_environment(monkeypatch):
    monkeypatch.setenv("MFG_FAULT", "launch:2")
    s = mfg.Server(1 << 40, slots=1, device=-1, max_group=1)  # reads MFG_FAULT
    monkeypatch.delenv("MFG_FAULT")
    try:
        tickets = [submit(s, 1024, 1024, 1024, "bf16") for _ in range(3)]
        res = wait_all(s, tickets)
    finally:
        _arm()
    assert [res[t]["status"] for t in tickets] == [0, capi.MFG_ERR_HIP, 0]
    s.close()


def test_large_requests_run_alone_on_separate_slots():
    s = mfg.Server(1 << 40, slots=4, device=-1, max_group=16)
    big = [submit(s, 8192, 8192, 8192, "f16") for _ in range(4)]  # 11 ms of dry-run time each
    small = [submit(s, 64, 64, 64, "f16") for _ in range(3)]
    res = wait_all(s, big + small)
    assert all(res[t]["group_size"] == 1 for t in big)
    assert len({res[t]["slot"] for t in big}) == 4
    assert s.stats()["max_concurrent_slots"] == 4
    # the small ones form one group of their own, never joined with a large one
    assert len({res[t]["t_start_ns"] for t in small}) == 1 and res[small[0]]["group_size"] == 3
    s.close()


def test_huge_k_never_joins_a_grouped_launch():
    # K > INT32_MAX does not fit the grouped kernel's work records
    s = mfg.Server(1 << 40, slots=1, device=-1, max_group=8)
    big = submit(s, 8192, 8192, 8192, "f16")
    small = [submit(s, 16, 16, 16, "f16") for _ in range(3)]
    K = (1 << 31) + 8
    huge = submit(s, 16, 16, K, "f16")
    res = wait_all(s, [big, huge] + small)
    assert res[huge]["status"] == 0 and res[huge]["group_size"] == 1
    assert all(res[t]["group_size"] == 3 for t in small)
    s.close()
