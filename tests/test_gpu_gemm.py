"""GPU parity of the GEMM modes against the FP64 oracle, through the C ABI.

Bar: |C - R_mode|_max <= 4 (K + 2) 2^-24 max(|alpha||A~||B~| + |beta||C0|)
(the 256^3 acceptance rule 4 K 2^-24 (|A||B|)_max extended to alpha, beta),
with R_mode the oracle's GEMM on exactly the operands the mode feeds the
matrix cores; and |C - R_exact| within the mode's a-priori accuracy bound.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, MODES, assert_parity, dev, host, need_gpu, run_gemm

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


# ------------------------------------------------------------- config 256^3
@pytest.mark.parametrize("mode", ["f32", "f16"])
def test_256_cube_acceptance(mode):
    """256^3, uniform[-1,1] from seed 0, alpha=1, beta=0; tolerance on rounded inputs."""
    A, B = workloads.uniform(0, [(256, 256), (256, 256)])
    C = run_gemm(mode, A, B)
    ref = oracle.reference(mode, A, B)
    assert_parity(C, ref, mode)
    # the literal acceptance rule 4*K*2^-24*(|A~||B~|)_max
    assert np.max(np.abs(C - ref.value)) <= 4 * 256 * 2.0 ** -24 * np.max(ref.absval)


# ------------------------------------------------- every mode, every config
RAGGED = [(300, 260, 200), (129, 65, 33), (512, 384, 320), (1000, 1000, 512), (257, 130, 384)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("shape", RAGGED)
def test_mode_parity_all_configs(mode, shape):
    M, N, K = shape
    A, B, C0 = workloads.normal(11, [(M, K), (K, N), (M, N)])
    ref = oracle.reference(mode, A, B, 1.25, -0.5, C0)
    ex = oracle.exact(A, B, 1.25, -0.5, C0)
    bound = oracle.representation_bound(mode, A, B, 1.25)
    outs = []
    for cfg in range(mfg.num_configs(mode)):
        try:
            C = run_gemm(mode, A, B, C0, 1.25, -0.5, config=cfg)
        except mfg.MfgError as e:
            # tiled FP32 kernels need 16-byte aligned rows (lda % 4 == 0); the fast
            # 16-bit kernels need K % 64 == 0 and N % 8 == 0; the tiled FP8
            # kernels K % 128 == 0; all report it
            name = mfg.config_name(mode, cfg)
            assert e.status == mfg.capi.MFG_ERR_UNSUPPORTED, name
            if mode == "fp8":
                assert name[0] == "p" and K % 128, name
            else:
                assert (mode == "f32" and cfg > 0 and (K % 4 or N % 4)) or (name[0] in "fpq" and (K % 64 or N % 8)), name
            continue
        err, tol = assert_parity(C, ref, f"{mode} cfg {cfg} {mfg.config_name(mode, cfg)}")
        # a-priori accuracy against the exact product
        assert np.all(np.abs(C - ex) <= bound + tol), f"{mode} cfg {cfg}: beyond the accuracy bound"
        outs.append(C)
    for cfg, C in enumerate(outs[1:], 1):
        assert np.array_equal(C.view(np.uint32), outs[0].view(np.uint32)), f"{mode}: cfg {cfg} not bitwise equal to cfg 0"


@pytest.mark.parametrize("mode", MODES)
def test_tiny_sizes_brute_force(mode):
    rng = np.random.default_rng(3)
    sizes = [1, 2, 3, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129]
    triples = [tuple(rng.choice(sizes, 3)) for _ in range(10)] + [(1, 1, 1), (17, 33, 15), (65, 1, 129)]
    for (M, N, K) in triples:
        A, B = workloads.uniform(int(M * 1000 + N * 10 + K), [(M, K), (K, N)])
        C = run_gemm(mode, A, B)
        assert_parity(C, oracle.reference(mode, A, B), f"{mode} {M}x{N}x{K}")


# ---------------------------------------------------------------- exactness
@pytest.mark.parametrize("mode", ["f32", "f16", "bf16", "split3", "fp8"])
def test_small_integers_exact(mode):
    """Integers |x| <= 8 are exact in every format; K=384 keeps sums < 2^24: exact."""
    A, B = workloads.small_ints(5, [(200, 384), (384, 136)])
    C = run_gemm(mode, A, B)
    assert np.array_equal(C.astype(np.float64), oracle.exact(A, B))


@pytest.mark.parametrize("mode", ["f16", "bf16", "f32"])
def test_identity_and_permutation(mode):
    n = 96
    (B,) = workloads.small_ints(6, [(n, 80)], -100, 100)
    I = np.eye(n, dtype=np.float32)
    assert np.array_equal(run_gemm(mode, I, B), B)
    perm = np.random.default_rng(1).permutation(n)
    P = np.zeros((n, n), np.float32)
    P[np.arange(n), perm] = 1
    assert np.array_equal(run_gemm(mode, P, B), B[perm])


# --------------------------------------------------------------- edge cases
def test_edges_zero_sizes_and_scalars():
    A, B, C0 = workloads.uniform(7, [(40, 24), (24, 56), (40, 56)])
    # K = 0: C = beta * C
    dC = dev(C0)
    mfg.gemm(dev(A[:, :0].copy()), dev(B[:0, :].copy()), dC, 1.0, 2.0, mode="f16", K=0)
    assert np.array_equal(host(dC), 2.0 * C0)
    # alpha = 0: C = beta * C (operands not read)
    dC = dev(C0)
    mfg.gemm(dev(A), dev(B), dC, 0.0, 0.5, mode="f16")
    assert np.array_equal(host(dC), 0.5 * C0)
    # beta = 0: NaN already in C does not propagate
    dC = torch.full((40, 56), float("nan"), device=DEV)
    mfg.gemm(dev(A), dev(B), dC, 1.0, 0.0, mode="f16")
    assert np.all(np.isfinite(host(dC)))
    # M = 0 and N = 0 are no-ops
    dC = dev(C0)
    st = mfg.lib().mfg_gemm(0, 56, 24, None, 24, dev(B).data_ptr(), 56, dC.data_ptr(), 56, 1.0, 0.0, 1, None)
    assert st == 0
    assert np.array_equal(host(dC), C0)


@pytest.mark.parametrize("mode", ["f16", "f32", "split3"])
def test_leading_dimensions_and_misalignment(mode):
    """ld > cols and operands starting one element into a buffer (unaligned)."""
    M, N, K = 70, 90, 50
    Abig, Bbig, Cbig = workloads.uniform(8, [(M, K + 13), (K, N + 7), (M, N + 5)])
    dA, dB, dC = dev(Abig), dev(Bbig), dev(Cbig)
    mfg.gemm(dA[:, 1:K + 1], dB[:, 1:N + 1], dC[:, 1:N + 1], 1.0, 1.0, mode=mode)
    C = host(dC)
    ref = oracle.reference(mode, Abig[:, 1:K + 1], Bbig[:, 1:N + 1], 1.0, 1.0, Cbig[:, 1:N + 1])
    assert_parity(C[:, 1:N + 1], ref, mode)
    assert np.array_equal(C[:, 0], Cbig[:, 0]) and np.array_equal(C[:, N + 1:], Cbig[:, N + 1:])


def test_invalid_arguments_enqueue_nothing():
    L = mfg.lib()
    A, B, C0 = workloads.uniform(9, [(8, 8), (8, 8), (8, 8)])
    dA, dB, dC = dev(A), dev(B), dev(C0)
    bad = [
        (8, 8, 8, dA.data_ptr(), 7, dB.data_ptr(), 8, dC.data_ptr(), 8, 1),   # lda < K
        (8, 8, 8, dA.data_ptr(), 8, dB.data_ptr(), 7, dC.data_ptr(), 8, 1),   # ldb < N
        (8, 8, 8, dA.data_ptr(), 8, dB.data_ptr(), 8, dC.data_ptr(), 7, 1),   # ldc < N
        (-1, 8, 8, dA.data_ptr(), 8, dB.data_ptr(), 8, dC.data_ptr(), 8, 1),  # negative size
        (8, 8, 8, None, 8, dB.data_ptr(), 8, dC.data_ptr(), 8, 1),            # null A
        (8, 8, 8, dA.data_ptr(), 8, dB.data_ptr(), 8, dC.data_ptr(), 8, 99),  # unknown mode
    ]
    for M, N, K, a, lda, b, ldb, c, ldc, mode in bad:
        assert L.mfg_gemm(M, N, K, a, lda, b, ldb, c, ldc, 1.0, 0.0, mode, None) == mfg.capi.MFG_ERR_INVALID_ARG
    assert np.array_equal(host(dC), C0)


# -------------------------------------------------- preconverted operands
@pytest.mark.parametrize("mode", ["f16", "bf16", "refine_a", "split3", "split4", "fp8", "bf16_split3"])
def test_preconverted_equals_fp32_input(mode):
    M, N, K = 260, 200, 300
    A, B = workloads.normal(10, [(M, K), (K, N)])
    C1 = run_gemm(mode, A, B)
    ldk = K + (-K) % 16
    ldn = N + (-N) % 16
    bufA = torch.zeros(mfg.convert_bytes(M, K, ldk, mode), dtype=torch.uint8, device=DEV)
    bufB = torch.zeros(mfg.convert_bytes(K, N, ldn, mode), dtype=torch.uint8, device=DEV)
    amode = mode
    bmode = "f16" if mode == "refine_a" else mode
    mfg.convert(dev(A), bufA, ldk, amode)
    mfg.convert(dev(B), bufB, ldn, bmode)
    dC = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    m = mfg.mode_of(mode) | mfg.MFG_IN_PRECONVERTED
    st = mfg.lib().mfg_gemm(M, N, K, bufA.data_ptr(), ldk, bufB.data_ptr(), ldn, dC.data_ptr(), N, 1.0, 0.0, m,
                            torch.cuda.current_stream().cuda_stream)
    assert st == 0
    assert np.array_equal(host(dC).view(np.uint32), C1.view(np.uint32))


# ------------------------------------------------------------ determinism
@pytest.mark.parametrize("mode", ["f16", "split3", "f32", "fp8"])
def test_run_to_run_bitwise(mode):
    A, B, C0 = workloads.normal(12, [(512, 512), (512, 512), (512, 512)])
    a, b = (run_gemm(mode, A, B, C0, 1.0, 1.0) for _ in range(2))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


# ------------------------------------------- leading dimension of 2^24 and up
def test_huge_leading_dimension_of_c():
    """ldc >= 2^24: the tiled kernels address a 32-row block of C with 32-bit
    offsets, so such C runs on the simple kernels (an explicit tiled
    configuration reports MFG_ERR_UNSUPPORTED) and the grouped kernel takes
    its 64-bit path; results stay within the parity bar."""
    M, N, K = 40, 72, 128
    ldc = (1 << 24) + 16
    A, B, C0 = workloads.uniform(13, [(M, K), (K, N), (M, N)])
    buf = torch.zeros((M - 1) * ldc + N, dtype=torch.float32, device=DEV)
    C = buf.as_strided((M, N), (ldc, 1))
    for mode in ("f16", "f32", "fp8"):
        C.copy_(dev(C0))
        mfg.gemm(dev(A), dev(B), C, 1.0, 1.0, mode=mode)
        assert_parity(host(C.contiguous()), oracle.reference(mode, A, B, 1.0, 1.0, C0), f"{mode} ldc=2^24+16")
        tiled = next(c for c in range(1, mfg.num_configs(mode)) if mfg.config_name(mode, c)[0] in "tfpq")
        with pytest.raises(mfg.MfgError) as e:
            mfg.gemm(dev(A), dev(B), C, 1.0, 1.0, mode=mode, config=tiled)
        assert e.value.status == mfg.capi.MFG_ERR_UNSUPPORTED
    dA, dB = dev(A).half(), dev(B).half()
    C.copy_(dev(C0))
    plan = mfg.GroupedPlan([(dA, dB, C)], mode="f16")
    plan.run(1.0, 1.0)
    ref = oracle.reference("f32", host(dA.float()), host(dB.float()), 1.0, 1.0, C0)
    assert_parity(host(C.contiguous()), ref, "grouped f16 ldc=2^24+16", mode="f16")
    plan.close()
    # the refined grouped kernel on the same C (head and residual planes)
    pa = torch.empty((2 * M, K), dtype=torch.float16, device=DEV)
    pb = torch.empty((2 * K, N), dtype=torch.float16, device=DEV)
    mfg.split_f16(dev(A), pa[:M], pa[M:])
    mfg.split_f16(dev(B), pb[:K], pb[K:])
    C.copy_(dev(C0))
    plan = mfg.GroupedPlan([(pa[:M], pb[:K], C)], mode="split3")
    plan.run(1.0, 1.0)
    assert_parity(host(C.contiguous()), oracle.reference("split3", A, B, 1.0, 1.0, C0), "grouped split3 ldc=2^24+16")
    plan.close()
    del C, buf
