"""GPU tests of the batched forms (paper Sec. IV.B: many small GEMMs at once).

Each problem of a batched or grouped launch must be bitwise identical to the
same problem run alone through mfg_gemm (all kernels share one accumulation
order), and within the parity tolerance of the oracle on sampled problems.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, assert_parity, dev, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _solo(mode, A, B, C0, alpha, beta, preconverted):
    C = C0.clone()
    mfg.gemm(A, B, C, alpha, beta, mode=mode, preconverted=preconverted)
    return C


@pytest.mark.parametrize("mode,shape,count", [
    ("f16", (16, 16, 16), 1000), ("bf16", (16, 16, 16), 333), ("f16", (17, 9, 100), 257), ("f16", (9, 13, 20), 101),
    ("f16", (64, 64, 64), 300), ("f16", (33, 70, 48), 65), ("bf16", (128, 100, 72), 37), ("f16", (129, 64, 64), 9),
    ("f16", (40, 50, 72), 77), ("bf16", (64, 20, 33), 45), ("f16", (20, 64, 200), 19), ("f16", (33, 33, 16), 8),
    ("f32", (16, 16, 16), 200), ("f32", (64, 64, 64), 50),
])
def test_batched_equals_solo_and_oracle(mode, shape, count):
    M, N, K = shape
    A32, B32, C0 = workloads.uniform(21, [(count, M, K), (count, K, N), (count, M, N)])
    if mode in ("f16", "bf16"):
        dt = torch.float16 if mode == "f16" else torch.bfloat16
        dA, dB = dev(A32).to(dt), dev(B32).to(dt)
    else:
        dA, dB = dev(A32), dev(B32)
    dC = dev(C0)
    mfg.gemm_batched(dA, dB, dC, 1.5, 0.5, mode=mode)
    got = host(dC)
    pre = mode != "f32"
    # every problem against its solo run (M, N <= 16 run two to an MFMA)
    for b in range(count):
        solo = host(_solo(mode, dA[b], dB[b], dev(C0[b]), 1.5, 0.5, pre))
        assert np.array_equal(got[b].view(np.uint32), solo.view(np.uint32)), f"problem {b} differs from solo"
        if b % 50 == 0 or b == count - 1:
            Ab = host(dA[b].float()).astype(np.float32)
            Bb = host(dB[b].float()).astype(np.float32)
            ref = oracle.reference("f32", Ab, Bb, 1.5, 0.5, C0[b])  # operands already rounded
            assert_parity(got[b], ref, f"{mode} problem {b}")


@pytest.mark.parametrize("count,size", [(65536, 16), (16384, 64), (1 << 18, 16)])
def test_batched_bench_workloads(count, size):
    """The benchmark's strided batches at their sizes (65536 x 16^3, 16384 x
    64^3, and the largest 16^3 batch of its sweep, 2^18), FP16 in, FP32 out,
    alpha = 1, beta = 0 over C filled with NaN (never read at beta = 0):
    every output finite, every 1024th problem and the last bitwise equal to
    its solo GEMM, every 8192nd and the last within the parity bar of the
    oracle."""
    A32, B32 = workloads.uniform(40 + size, [(count, size, size), (count, size, size)])
    dA, dB = dev(A32).half(), dev(B32).half()
    dC = torch.full((count, size, size), float("nan"), dtype=torch.float32, device=DEV)
    mfg.gemm_batched(dA, dB, dC, 1.0, 0.0, mode="f16")
    assert bool(torch.isfinite(dC).all())
    got = host(dC)
    for b in sorted(set(range(0, count, 1024)) | {count - 1}):
        solo = host(_solo("f16", dA[b], dB[b], torch.zeros_like(dC[b]), 1.0, 0.0, True))
        assert np.array_equal(got[b].view(np.uint32), solo.view(np.uint32)), f"problem {b} differs from solo"
    for b in sorted(set(range(0, count, 8192)) | {count - 1}):
        ref = oracle.reference("f16", A32[b], B32[b])
        assert_parity(got[b], ref, f"f16 batch {count}x{size}^3 problem {b}")


@pytest.mark.parametrize("mode,shape", [("split3", (16, 16, 40)), ("refine_a", (16, 16, 40)), ("split4", (16, 16, 40)),
                                        ("split3", (48, 64, 40)), ("split4", (64, 40, 72)),
                                        ("bf16_split3", (16, 16, 40)), ("bf16_split3", (48, 64, 40))])
def test_batched_refined_equals_solo(mode, shape):
    count, (M, N, K) = 96, shape
    A, B, C0 = workloads.normal(22, [(count, M, K), (count, K, N), (count, M, N)])
    dC = dev(C0)
    mfg.gemm_batched(dev(A), dev(B), dC, 1.0, 1.0, mode=mode)
    got = host(dC)
    for b in (0, 1, 47, 95):
        solo = np.copy(C0[b])
        d = dev(solo)
        mfg.gemm(dev(A[b]), dev(B[b]), d, 1.0, 1.0, mode=mode)
        assert np.array_equal(got[b].view(np.uint32), host(d).view(np.uint32))
        assert_parity(got[b], oracle.reference(mode, A[b], B[b], 1.0, 1.0, C0[b]), f"{mode} problem {b}")


def _grouped_problems(count, lo, hi, seed, unaligned_every=0):
    dims = workloads.loguniform_dims(seed, count, lo, hi)
    probs, host_ops = [], []
    for i, (m, n, k) in enumerate(dims):
        m, n, k = int(m), int(n), int(k)
        if unaligned_every and i % unaligned_every == 0:
            lda, ldb = k, n  # unaligned leading dimensions -> per-wave tile path
        else:
            lda, ldb = -(-k // 8) * 8, -(-n // 8) * 8
        A, B = workloads.uniform(1000 + i, [(m, lda), (k, ldb)])
        fa, fb = dev(A).half(), dev(B).half()
        fa[:, k:] = float("nan")  # row padding never reaches a result
        fb[:, n:] = float("nan")
        dA, dB = fa[:, :k], fb[:, :n]
        dC = torch.zeros((m, n), dtype=torch.float32, device=DEV)
        probs.append((dA, dB, dC))
        host_ops.append((A[:, :k], B[:, :n]))
    return probs, host_ops


def test_grouped_equals_solo_and_graph_replays():
    probs, host_ops = _grouped_problems(300, 16, 200, 6, unaligned_every=7)
    plan = mfg.GroupedPlan(probs, "f16")
    info = plan.info()
    # one work item per 128 x 128 output tile
    assert info["work_items"] == sum(-(-p[0].shape[0] // 128) * -(-p[1].shape[1] // 128) for p in probs)
    plan.run(1.0, 0.0)
    first = [host(p[2]).copy() for p in probs]
    for i in range(300):
        A, B, C = probs[i]
        solo = torch.zeros_like(C)
        mfg.gemm(A, B, solo, 1.0, 0.0, mode="f16", preconverted=True)
        assert np.array_equal(first[i].view(np.uint32), host(solo).view(np.uint32)), f"problem {i}"
        if i % 23 == 0:
            a16 = oracle.f16_round(host_ops[i][0]).astype(np.float32)
            b16 = oracle.f16_round(host_ops[i][1]).astype(np.float32)
            assert_parity(first[i], oracle.reference("f32", a16, b16), f"grouped problem {i}")
    # alpha and beta: C = 0.75 A B - 0.5 C, against the solo GEMM on the same C
    c0 = [torch.randn_like(p[2]) for p in probs]
    for p, c in zip(probs, c0):
        p[2].copy_(c)
    plan.run(0.75, -0.5)
    for i in range(0, 300, 3):
        A, B, C = probs[i]
        solo = c0[i].clone()
        mfg.gemm(A, B, solo, 0.75, -0.5, mode="f16", preconverted=True)
        assert np.array_equal(host(C).view(np.uint32), host(solo).view(np.uint32)), f"beta problem {i}"
    # graph replays with eager work in between; every replay must equal the eager result
    for rep in range(3):
        for p in probs:
            p[2].fill_(float("nan"))
        plan.graph_launch(1.0, 0.0)
        junk = torch.randn(512, 512, device=DEV) @ torch.randn(512, 512, device=DEV)  # unrelated eager work
        torch.cuda.synchronize()
        del junk
        for i in range(0, 300, 11):
            assert np.array_equal(host(probs[i][2]).view(np.uint32), first[i].view(np.uint32)), f"replay {rep} problem {i}"
    plan.close()


def test_grouped_large_operand_ld_equals_solo():
    """Aligned problems with lda or ldb >= 2^22 go to the element-wise work list
    (the aligned kernel addresses its pieces with 32-bit offsets): each is
    bitwise equal to its solo run, beside ordinary problems in the same plan."""
    big = (1 << 22) + 8
    specs = [(3, 40, 24, big, None), (70, 33, 5, None, big), (130, 136, 72, None, None), (9, 17, 100, None, None)]
    probs = []
    for i, (m, n, k, lda, ldb) in enumerate(specs):
        A, B = workloads.uniform(4000 + i, [(m, k), (k, n)])
        a = torch.zeros((m, lda or -(-k // 8) * 8), dtype=torch.float16, device=DEV)
        b = torch.zeros((k, ldb or -(-n // 8) * 8), dtype=torch.float16, device=DEV)
        a[:, :k] = dev(A).half()
        b[:, :n] = dev(B).half()
        probs.append((a[:, :k], b[:, :n], torch.zeros((m, n), dtype=torch.float32, device=DEV)))
    plan = mfg.GroupedPlan(probs, "f16")
    plan.run(1.0, 0.0)
    for i, (a, b, c) in enumerate(probs):
        solo = torch.zeros_like(c)
        mfg.gemm(a, b, solo, 1.0, 0.0, mode="f16", preconverted=True)
        assert np.array_equal(host(c).view(np.uint32), host(solo).view(np.uint32)), f"problem {specs[i]}"
    plan.close()


def test_grouped_rejects_unsupported_mode():
    probs, _ = _grouped_problems(4, 16, 64, 9)
    for mode in ("f32", "fp8"):
        with pytest.raises(mfg.MfgError):
            mfg.GroupedPlan(probs, mode)


def _planes(X32, ld, two):
    """X (FP32, rows x cols) in the refined storage form: head plane, then
    (two) the scaled residual plane at +rows*ld; padding columns are NaN."""
    rows, cols = X32.shape
    P = torch.full((2 * rows if two else rows, ld), float("nan"), dtype=torch.float16, device=DEV)
    X = dev(X32)
    if two:
        mfg.split_f16(X, P[:rows, :cols], P[rows:, :cols])
    else:
        mfg.round_f16(X, P[:rows, :cols])
    return P[:rows, :cols]


@pytest.mark.parametrize("mode", ["refine_a", "split3", "split4"])
def test_grouped_refined_equals_solo_and_oracle(mode):
    """The refined modes (Eq. 1, Eq. 2) in the grouped persistent kernel: every
    problem bitwise equal to mfg_gemm on it alone (preconverted planes), sampled
    problems within the parity bar of the oracle's mode-faithful reference."""
    count = 120
    dims = workloads.loguniform_dims(31, count, 16, 300)
    probs, ops = [], []
    for i, (m, n, k) in enumerate(dims):
        m, n, k = int(m), int(n), int(k)
        lda, ldb = (k, n) if i % 9 == 0 else (-(-k // 8) * 8, -(-n // 8) * 8)
        A, B, C0 = workloads.normal(2000 + i, [(m, k), (k, n), (m, n)])
        dA = _planes(A, lda, True)
        dB = _planes(B, ldb, mode != "refine_a")
        probs.append((dA, dB, dev(C0)))
        ops.append((A, B, C0))
    plan = mfg.GroupedPlan(probs, mode)
    info = plan.info()
    npa, npb = 2, (1 if mode == "refine_a" else 2)
    exp_bytes = sum(2 * (npa * a.shape[0] * a.shape[1] + npb * b.shape[0] * b.shape[1]) + 4 * a.shape[0] * b.shape[1]
                    for a, b, _ in ops)
    assert info["bytes"] == pytest.approx(exp_bytes)
    plan.run(1.25, -0.5)
    for i, (dA, dB, dC) in enumerate(probs):
        A, B, C0 = ops[i]
        solo = dev(C0)
        mfg.gemm(dA, dB, solo, 1.25, -0.5, mode=mode, preconverted=True)
        assert np.array_equal(host(dC).view(np.uint32), host(solo).view(np.uint32)), f"{mode} problem {i}"
        if i % 17 == 0:
            assert_parity(host(dC), oracle.reference(mode, A, B, 1.25, -0.5, C0), f"{mode} grouped problem {i}")
    # graph replays, each equal to the eager run
    first = [host(p[2]).copy() for p in probs]
    for rep in range(2):
        for (dA, dB, dC), (_, _, C0) in zip(probs, ops):
            dC.copy_(dev(C0))
        plan.graph_launch(1.25, -0.5)
        torch.cuda.synchronize()
        for i in range(0, count, 7):
            assert np.array_equal(host(probs[i][2]).view(np.uint32), first[i].view(np.uint32)), f"replay {rep} {i}"
    plan.close()


@pytest.mark.parametrize("mode", ["f16", "split3"])
def test_grouped_bench_workload_4096(mode):
    """The benchmark's grouped workload at its size: 4096 problems with M, N, K
    log-uniform in [16, 512] (dimension seed 6, ld rounded up to 8), one graph
    launch of the plan, alpha = 1, beta = 0 over C filled with NaN (never read
    at beta = 0).  Every 16th problem bitwise equal to its solo GEMM; every
    128th and the largest within the parity bar of the oracle's reference."""
    count = 4096
    dims = workloads.loguniform_dims(6, count, 16, 512)
    two = mode != "f16"
    probs, ops = [], []
    for i, (m, n, k) in enumerate(dims):
        m, n, k = int(m), int(n), int(k)
        A, B = workloads.uniform(7000 + i, [(m, k), (k, n)])
        dA, dB = _planes(A, -(-k // 8) * 8, two), _planes(B, -(-n // 8) * 8, two)
        probs.append((dA, dB, torch.full((m, n), float("nan"), dtype=torch.float32, device=DEV)))
        ops.append((A, B))
    plan = mfg.GroupedPlan(probs, mode)
    plan.graph_launch(1.0, 0.0)
    torch.cuda.synchronize()
    print(f"grouped {mode}: {count} problems, {plan.info()['work_items']} work items", flush=True)
    for i in range(0, count, 16):
        dA, dB, dC = probs[i]
        solo = torch.zeros_like(dC)
        mfg.gemm(dA, dB, solo, 1.0, 0.0, mode=mode, preconverted=True)
        assert np.array_equal(host(dC).view(np.uint32), host(solo).view(np.uint32)), f"{mode} problem {i}"
    sizes = [a.shape[0] * a.shape[1] * b.shape[1] for a, b in ops]
    for i in sorted(set(range(0, count, 128)) | {int(np.argmax(sizes))}):
        A, B = ops[i]
        assert_parity(host(probs[i][2]), oracle.reference(mode, A, B), f"{mode} grouped problem {i}")
    plan.close()


@pytest.mark.parametrize("mode", ["refine_a", "split4"])
def test_grouped_refined_degenerate_shapes(mode):
    """Empty, single-row/column, K = 0 and tile-edge problems in one refined
    grouped plan, each bitwise equal to its solo run."""
    shapes = [(1, 1, 1), (0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 130, 3), (130, 1, 65), (64, 64, 64), (65, 65, 129),
              (3, 200, 8), (200, 3, 9)]
    probs, c0 = [], []
    for i, (m, n, k) in enumerate(shapes):
        A, B, C0 = workloads.normal(3000 + i, [(m, k), (k, n), (m, n)])
        dA = _planes(A, max(8, -(-k // 8) * 8), True)
        dB = _planes(B, max(8, -(-n // 8) * 8), mode != "refine_a")
        probs.append((dA, dB, dev(C0)))
        c0.append(C0)
    plan = mfg.GroupedPlan(probs, mode)
    plan.run(0.5, 2.0)
    for i, (dA, dB, dC) in enumerate(probs):
        solo = dev(c0[i])
        mfg.gemm(dA, dB, solo, 0.5, 2.0, mode=mode, preconverted=True)
        assert np.array_equal(host(dC).view(np.uint32), host(solo).view(np.uint32)), f"{mode} shape {shapes[i]}"
    plan.close()


@pytest.mark.parametrize("mode", ["f16", "bf16", "refine_a", "split3", "split4", "bf16_split3"])
def test_grouped_fp32_input_equals_solo(mode):
    """MFG_IN_FP32 plans: one conversion launch over every problem's FP32 A and
    B into plan-owned storage, then the grouped kernel.  Every problem bitwise
    equal to mfg_gemm on its FP32 operands alone (unaligned and padded
    operands, tiny and empty problems included), graph replays equal to the
    eager run, and the plan's byte count including the conversion pass."""
    dims = [tuple(int(x) for x in d) for d in workloads.loguniform_dims(43, 90, 1, 300)]
    dims += [(0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 1, 1)]
    probs, c0 = [], []
    for i, (m, n, k) in enumerate(dims):
        A, B, C0 = workloads.normal(4000 + i, [(m, k + 3), (k, n + 5), (m, n)])
        dA, dB = dev(A), dev(B)
        if i % 4 == 0:  # one element into the buffer: rows not 16-byte aligned
            dA, dB = dA[:, 1:k + 1], dB[:, 2:n + 2]
        else:
            dA, dB = dA[:, :k], dB[:, :n]
        probs.append((dA, dB, dev(C0)))
        c0.append(C0)
    plan = mfg.GroupedPlan(probs, mode, fp32_in=True)
    npa = 1 if mode in ("f16", "bf16") else 2
    npb = 2 if mode in ("split3", "split4", "bf16_split3") else 1
    exp = sum(4 * (m * k + k * n) + 2 * (npa * m * k + npb * k * n) + 2 * (npa * m * k + npb * k * n) + 4 * m * n
              for (m, n, k) in dims)
    assert plan.info()["bytes"] == pytest.approx(exp)
    plan.run(0.75, 0.5)
    first = [host(p[2]).copy() for p in probs]
    for i, (dA, dB, dC) in enumerate(probs):
        solo = dev(c0[i])
        mfg.gemm(dA, dB, solo, 0.75, 0.5, mode=mode)
        assert np.array_equal(first[i].view(np.uint32), host(solo).view(np.uint32)), f"{mode} problem {i} {dims[i]}"
    for rep in range(2):
        for (dA, dB, dC), C0 in zip(probs, c0):
            dC.copy_(dev(C0))
        plan.graph_launch(0.75, 0.5)
        torch.cuda.synchronize()
        for i in range(0, len(probs), 5):
            assert np.array_equal(host(probs[i][2]).view(np.uint32), first[i].view(np.uint32)), f"replay {rep} {i}"
    plan.close()


@pytest.mark.parametrize("mode", ["refine_a", "split3", "split4", "bf16_split3"])
def test_batched_refined_preconverted_equals_fp32_input(mode):
    """MFG_IN_PRECONVERTED on a refined batch: entry b's head plane at
    A + b*strideA and its residual plane M*lda later (as mfg_convert writes
    them) give the same bits as the batch from FP32 operands."""
    count, M, N, K = 40, 48, 72, 60
    A, B, C0 = workloads.normal(23, [(count, M, K), (count, K, N), (count, M, N)])
    dC = dev(C0)
    mfg.gemm_batched(dev(A), dev(B), dC, 1.25, -0.5, mode=mode)
    ldk, ldn = 64, 72
    two_b = mode != "refine_a"
    pa = torch.zeros((count, 2 * M, ldk), dtype=torch.int16, device=DEV)
    pb = torch.zeros((count, (2 if two_b else 1) * K, ldn), dtype=torch.int16, device=DEV)
    for b in range(count):
        mfg.convert(dev(A[b]), pa[b], ldk, mode)
        mfg.convert(dev(B[b]), pb[b], ldn, mode if two_b else "f16")
    dP = dev(C0)
    mfg.gemm_batched(pa, pb, dP, 1.25, -0.5, mode=mode, preconverted=True, M=M, K=K)
    assert np.array_equal(host(dP).view(np.uint32), host(dC).view(np.uint32))
    assert_parity(host(dP)[7], oracle.reference(mode, A[7], B[7], 1.25, -0.5, C0[7]), f"{mode} entry 7")
