"""mfg_gemm_noalloc: the allocation-free variant of mfg_gemm (operands
converted into the library's fixed per-device array instead of a workspace
grown with hipMalloc).  Through the C ABI, every mode's result must be
bitwise that of mfg_gemm on the same arguments, on two calls in a row (the
second smaller, so it runs over what the first left in the array); a call
that needs more than the array holds is refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, dev, host, need_gpu

pytestmark = pytest.mark.gpu

MODES = ["f16", "bf16", "refine_a", "split3", "split4", "bf16_split3", "bf16_split6", "fp8", "f32"]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _call(fn, A, B, C, alpha, beta, mode):
    M, K = A.shape
    N = B.shape[1]
    st = getattr(mfg.lib(), fn)(M, N, K, ctypes.c_void_p(A.data_ptr()), A.stride(0), ctypes.c_void_p(B.data_ptr()),
                                B.stride(0), ctypes.c_void_p(C.data_ptr()), C.stride(0), alpha, beta,
                                mfg.capi.MODE_BY_NAME[mode],
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("mode", MODES)
def test_noalloc_equals_gemm_on_two_calls(mode):
    for i, (M, N, K) in enumerate([(700, 520, 640), (129, 65, 200)]):  # second call smaller
        A, B, C0 = workloads.normal(40 + i, [(M, K), (K, N), (M, N)])
        dA, dB = dev(A), dev(B)
        c_ref, c_new = dev(C0), dev(C0)
        assert _call("mfg_gemm", dA, dB, c_ref, 1.25, -0.5, mode) == 0
        assert _call("mfg_gemm_noalloc", dA, dB, c_new, 1.25, -0.5, mode) == 0
        assert np.array_equal(host(c_new).view(np.uint32), host(c_ref).view(np.uint32)), (mode, M, N, K)


def test_noalloc_headline_fp8_tiles_and_repeat():
    # a size the FP8 tiled kernels take (K % 128 == 0), then the same call again
    M, N, K = 1024, 768, 1024
    A, B = workloads.uniform(44, [(M, K), (K, N)])
    dA, dB = dev(A), dev(B)
    ref = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    assert _call("mfg_gemm", dA, dB, ref, 1.0, 0.0, "fp8") == 0
    for _ in range(2):
        c = torch.full((M, N), float("nan"), dtype=torch.float32, device=DEV)
        assert _call("mfg_gemm_noalloc", dA, dB, c, 1.0, 0.0, "fp8") == 0
        assert np.array_equal(host(c).view(np.uint32), host(ref).view(np.uint32))


def test_noalloc_refuses_more_than_the_array_before_running():
    # FP16 from FP32: 2 * (M*K + K*N) bytes of converted operands > 64 MiB
    M = N = K = 4608
    dA = torch.zeros((M, K), dtype=torch.float32, device=DEV)
    dB = torch.zeros((K, N), dtype=torch.float32, device=DEV)
    c = torch.full((M, N), 3.0, dtype=torch.float32, device=DEV)
    assert _call("mfg_gemm_noalloc", dA, dB, c, 1.0, 0.0, "f16") == mfg.capi.MFG_ERR_UNSUPPORTED
    assert bool(torch.all(c == 3.0))
    # preconverted operands need no array: served at any size
    a16 = torch.zeros((M, K), dtype=torch.float16, device=DEV)
    b16 = torch.zeros((K, N), dtype=torch.float16, device=DEV)
    st = mfg.lib().mfg_gemm_noalloc(M, N, K, ctypes.c_void_p(a16.data_ptr()), K, ctypes.c_void_p(b16.data_ptr()), N,
                                    ctypes.c_void_p(c.data_ptr()), N, 1.0, 0.0,
                                    mfg.capi.MFG_F16 | mfg.capi.MFG_IN_PRECONVERTED,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0 and bool(torch.all(c == 0.0))
