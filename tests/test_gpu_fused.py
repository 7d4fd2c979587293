"""The refined GEMMs straight from FP32 operands (the split fused into the
operand staging): bitwise the two-pass result (split pass, then the GEMM on
the planes) for every refined mode it serves, at the parity bar against the
oracle, with no workspace; the shapes it does not serve report it."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, assert_parity, dev, host, need_gpu, run_gemm

pytestmark = pytest.mark.gpu
MODES = ["refine_a", "split3", "bf16_split3"]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _fused(mode):
    n = mfg.num_configs(mode)
    cfg = n - 1
    assert mfg.config_name(mode, cfg).startswith("fused")
    return cfg


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("shape", [(128, 128, 64), (300, 264, 192), (512, 384, 320), (1000, 1000, 512),
                                   (129, 8, 128), (64, 520, 1024), (129, 12, 128), (300, 260, 192), (7, 4, 64)])
def test_fused_bitwise_equals_two_pass(mode, shape):
    M, N, K = shape
    A, B, C0 = workloads.normal(51, [(M, K), (K, N), (M, N)])
    two = run_gemm(mode, A, B, C0, 1.25, -0.5, config=0)
    fused = run_gemm(mode, A, B, C0, 1.25, -0.5, config=_fused(mode))
    assert np.array_equal(fused.view(np.uint32), two.view(np.uint32)), (mode, shape)
    assert_parity(fused, oracle.reference(mode, A, B, 1.25, -0.5, C0), f"{mode} fused {shape}")


@pytest.mark.parametrize("mode", MODES)
def test_fused_wide_range_and_strided_operands(mode):
    """sign * 2^u inputs (u in [-12, 12]: heads and residuals across the FP16
    range) in sub-blocks of larger arrays (lda, ldb, ldc beyond the sizes)."""
    M, N, K = 200, 136, 256
    g = np.random.default_rng(52)
    big_a = (np.where(g.random((M + 7, K + 12)) < 0.5, -1, 1) * np.ldexp(1.0, g.integers(-12, 13, (M + 7, K + 12)))
             * g.uniform(1, 2, (M + 7, K + 12))).astype(np.float32)
    big_b = g.standard_normal((K + 3, N + 24)).astype(np.float32)
    dA, dB = dev(big_a), dev(big_b)
    a, b = dA[3:3 + M, 4:4 + K], dB[1:1 + K, 8:8 + N]  # 16-byte aligned starts, ld % 4 == 0
    cbuf = torch.zeros((M, N + 40), dtype=torch.float32, device=DEV)
    outs = []
    for cfg in (0, _fused(mode)):
        c = cbuf[:, 16:16 + N]
        c.zero_()
        mfg.gemm(a, b, c, 1.0, 0.0, mode=mode, config=cfg)
        outs.append(host(c.contiguous()))
    assert np.array_equal(outs[1].view(np.uint32), outs[0].view(np.uint32))
    A, B = big_a[3:3 + M, 4:4 + K], big_b[1:1 + K, 8:8 + N]
    assert_parity(outs[1], oracle.reference(mode, A, B), f"{mode} fused strided")


def test_fused_unserved_shapes_report_unsupported():
    cfg = _fused("split3")
    for (M, N, K) in [(64, 64, 100), (64, 62, 128), (64, 2, 128)]:  # K % 64, N % 4, N < 4
        A, B = workloads.uniform(53, [(M, K), (K, N)])
        with pytest.raises(mfg.MfgError) as e:
            run_gemm("split3", A, B, config=cfg)
        assert e.value.status == mfg.capi.MFG_ERR_UNSUPPORTED
    # preconverted planes: the fused kernels read FP32 operands
    a16 = torch.zeros((128, 128), dtype=torch.float16, device=DEV)
    c = torch.zeros((64, 64), dtype=torch.float32, device=DEV)
    with pytest.raises(mfg.MfgError) as e:
        mfg.gemm(a16, a16, c, mode="split3", preconverted=True, M=64, K=64, config=cfg)
    assert e.value.status == mfg.capi.MFG_ERR_UNSUPPORTED


def test_fused_tuned_entry_and_allocation_free_fallback():
    """A tuned table entry naming the fused kernel is what mfg_gemm runs; the
    allocation-free entry point serves a refined mode beyond its array with
    the fused kernel (which needs none)."""
    L = mfg.lib()
    M = N = K = 3072  # two-pass SPLIT3 would convert 4 * 2 * 3072^2 bytes = 72 MiB > 64 MiB
    A, B = workloads.uniform(54, [(M, K), (K, N)])
    dA, dB = dev(A), dev(B)
    cfg = _fused("split3")
    ref = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    mfg.gemm(dA, dB, ref, mode="split3", config=cfg)
    m = mfg.capi.MFG_F16_SPLIT3
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    c = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    args = (M, N, K, ctypes.c_void_p(dA.data_ptr()), K, ctypes.c_void_p(dB.data_ptr()), N,
            ctypes.c_void_p(c.data_ptr()), N, 1.0, 0.0, m, s)
    L.mfg_tune_clear()
    try:
        assert L.mfg_gemm_noalloc(*args) == 0  # two-pass planes: beyond the array
        assert np.array_equal(host(c).view(np.uint32), host(ref).view(np.uint32))
        import tempfile, os
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "t.txt")
            with open(path, "w") as f:
                f.write(f"{m} 11 11 11 {cfg}\n")
            assert L.mfg_tune_load(path.encode()) == 0
        assert L.mfg_tune_lookup(M, N, K, m) == cfg
        c2 = torch.zeros((M, N), dtype=torch.float32, device=DEV)
        mfg.gemm(dA, dB, c2, mode="split3")  # the tuned entry: the fused kernel
        assert np.array_equal(host(c2).view(np.uint32), host(ref).view(np.uint32))
    finally:
        L.mfg_tune_clear()
