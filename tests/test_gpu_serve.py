"""GPU tests of the serving loop (mfg_server_*): a mixed stream of requests of
all modes and uneven sizes, operands taken as sub-blocks of resident FP32
pools, served with continuous batching under an HBM budget.

Every request's result must be bitwise identical to the same request run
alone through mfg_gemm (the alone-vs-mix guarantee), and sampled requests
must be within the parity tolerance of the oracle's mode-faithful reference.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, MODES, assert_parity, dev, host, need_gpu

pytestmark = pytest.mark.gpu

POOL = 768


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _pools(seed):
    A, B = workloads.normal(seed, [(POOL, POOL), (POOL, POOL)])
    return A, B, dev(A), dev(B)


def _requests(seed, n, lo, hi):
    g = np.random.default_rng(seed)
    dims = workloads.loguniform_dims(seed, n, lo, hi)
    reqs = []
    for i, (M, N, K) in enumerate(dims):
        M, N, K = int(M), int(N), int(K)
        ar, ac = (int(x) for x in g.integers(0, POOL - np.array([M, K]) + 1))
        br, bc = (int(x) for x in g.integers(0, POOL - np.array([K, N]) + 1))
        alpha, beta = [(1.0, 0.0), (1.5, 0.5), (-0.75, 1.0)][i % 3]
        reqs.append(dict(M=M, N=N, K=K, mode=MODES[i % len(MODES)], a=(ar, ac), b=(br, bc), alpha=alpha, beta=beta,
                         C0=g.uniform(-1, 1, size=(M, N)).astype(np.float32)))
    return reqs


def _wait(server, tickets, timeout=120.0):
    done, t0 = {}, time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            st, r = server.poll(t)
            if st != mfg.capi.MFG_PENDING:
                r["status"] = st
                done[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.0005)
    return done


def _serve_and_check(reqs, budget, slots, max_group, seed, blocker=False):
    A, B, dA, dB = _pools(seed)
    outs = []
    for r in reqs:
        (ar, ac), (br, bc) = r["a"], r["b"]
        outs.append((dA[ar:ar + r["M"], ac:ac + r["K"]], dB[br:br + r["K"], bc:bc + r["N"]], dev(r["C0"])))
    if blocker:  # an FP32 8192^3 request (~10 ms) that holds the only slot while the rest queue up
        big = [torch.ones((8192, 8192), device=DEV) for _ in range(3)]
    torch.cuda.synchronize()  # the server's streams do not order after torch's
    server = mfg.Server(budget, slots=slots, max_group=max_group)
    first = [server.submit(big[0], big[1], big[2], "f32")] if blocker else []
    tickets = [server.submit(a, b, c, r["mode"], r["alpha"], r["beta"]) for r, (a, b, c) in zip(reqs, outs)]
    res = _wait(server, first + tickets)
    stats = server.stats()
    server.close()
    torch.cuda.synchronize()
    for i, (r, (a, b, c), t) in enumerate(zip(reqs, outs, tickets)):
        assert res[t]["status"] == 0, (i, r["mode"], res[t])
        alone = dev(r["C0"])
        mfg.gemm(a, b, alone, r["alpha"], r["beta"], mode=r["mode"])
        got = host(c)
        assert np.array_equal(got.view(np.uint32), host(alone).view(np.uint32)), \
            f"request {i} ({r['mode']}, {r['M']}x{r['N']}x{r['K']}, group {res[t]['group_size']}) differs from alone"
        if i % 4 == 0:
            (ar, ac), (br, bc) = r["a"], r["b"]
            An = A[ar:ar + r["M"], ac:ac + r["K"]]
            Bn = B[br:br + r["K"], bc:bc + r["N"]]
            ref = oracle.reference(r["mode"], An, Bn, r["alpha"], r["beta"], r["C0"])
            assert_parity(got, ref, f"{r['mode']} request {i}", mode=r["mode"])
        x = res[t]
        assert x["t_submit_ns"] <= x["t_admit_ns"] <= x["t_start_ns"] <= x["t_end_ns"]
    return res, stats


def test_mixed_trace_alone_vs_mix_and_oracle():
    reqs = _requests(11, 84, 16, 640)
    res, stats = _serve_and_check(reqs, budget=1 << 30, slots=1, max_group=8, seed=12, blocker=True)
    assert stats["completed"] == len(reqs) + 1 and stats["failed"] == 0
    assert max(r["group_size"] for r in res.values()) >= 2  # requests queued behind the blocker were batched
    assert stats["launches"] < len(reqs)


def test_mixed_trace_on_concurrent_slots():
    reqs = _requests(17, 60, 16, 700)
    res, stats = _serve_and_check(reqs, budget=1 << 30, slots=4, max_group=8, seed=18)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert {r["slot"] for r in res.values()} <= {0, 1, 2, 3}


def test_tight_budget_admission_on_gpu():
    reqs = _requests(13, 40, 64, 700)
    budget = 6 << 20  # a few requests' converted operands at a time
    res, stats = _serve_and_check(reqs, budget=budget, slots=3, max_group=4, seed=14)
    assert stats["peak_bytes_in_use"] <= budget
    assert stats["bytes_in_use"] == 0
    assert stats["max_concurrent_slots"] <= 3


def test_degenerate_requests_on_gpu():
    A, B, dA, dB = _pools(15)
    server = mfg.Server(1 << 28, slots=2, max_group=4)
    c0 = dev(np.full((5, 7), 2.0, np.float32))
    c1 = dev(np.full((3, 4), np.nan, np.float32))
    torch.cuda.synchronize()
    t1 = server.submit(dA[:5, :0], dB[:0, :7], c0, "split3", 1.0, 0.5)           # K = 0: C = beta C
    t2 = server.submit(dA[:3, :16], dB[:16, :4], c1, "fp8", 1.0, 0.0)             # beta = 0: C not read
    res = _wait(server, [t1, t2])
    server.close()
    assert res[t1]["status"] == 0 and res[t2]["status"] == 0
    assert np.all(host(c0) == 1.0)
    assert np.all(np.isfinite(host(c1)))


def test_small_requests_overlap_a_long_one():
    """Continuous batching on the device: with four slots, small requests that
    arrive while a long request runs are admitted onto the free slots and
    finish before it; each result is bitwise that of the request alone."""
    A, B, dA, dB = _pools(21)
    big = [torch.ones((8192, 8192), device=DEV) for _ in range(3)]  # FP32 8192^3: ~9 ms alone
    reqs = _requests(22, 12, 64, 384)
    views = []
    for r in reqs:
        (ar, ac), (br, bc) = r["a"], r["b"]
        views.append((dA[ar:ar + r["M"], ac:ac + r["K"]], dB[br:br + r["K"], bc:bc + r["N"]], dev(r["C0"])))
    torch.cuda.synchronize()
    server = mfg.Server(1 << 30, slots=4, max_group=4)
    tb = server.submit(big[0], big[1], big[2], "f32")
    time.sleep(0.002)  # the long request is on the device
    tickets = [server.submit(a, b, c, r["mode"], r["alpha"], r["beta"]) for r, (a, b, c) in zip(reqs, views)]
    res = _wait(server, [tb] + tickets)
    stats = server.stats()
    server.close()
    assert res[tb]["status"] == 0
    assert stats["max_concurrent_slots"] >= 2
    early = [t for t in tickets if res[t]["t_end_ns"] < res[tb]["t_end_ns"]]
    assert len(early) >= len(tickets) // 2, "small requests waited for the long one"
    for i, (r, (a, b, c), t) in enumerate(zip(reqs, views, tickets)):
        assert res[t]["status"] == 0
        if t in early:
            assert res[t]["slot"] != res[tb]["slot"]
        alone = dev(r["C0"])
        mfg.gemm(a, b, alone, r["alpha"], r["beta"], mode=r["mode"])
        assert np.array_equal(host(c).view(np.uint32), host(alone).view(np.uint32)), f"request {i} ({r['mode']})"


def test_injected_launch_fault_fails_one_request_on_gpu():
    """A launch failure (injected on the host: the GEMM is not launched) marks
    that request failed; the server keeps serving and every other result is
    bitwise that of the request alone."""
    A, B, dA, dB = _pools(23)
    shapes = [(600, 520, 256), (640, 520, 320), (520, 600, 128), (700, 512, 192)]  # not grouped: one launch each
    views = [(dA[:m, :k], dB[:k, :n], dev(np.zeros((m, n), np.float32))) for m, n, k in shapes]
    torch.cuda.synchronize()
    server = mfg.Server(1 << 30, slots=1, max_group=1)
    assert mfg.lib().mfg_fault_inject(2, 0) == 0
    try:
        tickets = []
        for a, b, c in views:  # one at a time: launches happen in submission order
            tickets.append(server.submit(a, b, c, "split3"))
            server.drain()
        res = _wait(server, tickets)
    finally:
        mfg.lib().mfg_fault_inject(0, 0)
    stats = server.stats()
    server.close()
    assert [res[t]["status"] for t in tickets] == [0, mfg.capi.MFG_ERR_HIP, 0, 0]
    assert stats["failed"] == 1 and stats["completed"] == 3 and stats["bytes_in_use"] == 0
    for i, ((a, b, c), t) in enumerate(zip(views, tickets)):
        if i == 1:
            continue
        alone = torch.zeros_like(c)
        mfg.gemm(a, b, alone, 1.0, 0.0, mode="split3")
        assert np.array_equal(host(c).view(np.uint32), host(alone).view(np.uint32))
