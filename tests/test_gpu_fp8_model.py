"""Pins the accumulation behaviour of the gfx950 E4M3 matrix instruction, as
seen through the library's FP8 mode (preconverted codes, tile scales 1).

The instruction multiplies E4M3 codes exactly but does not add its 64
products exactly in FP32 (448 + 2^-9 comes back as 448).  Measured over
random codes its error stays below 2^-12 of the sum of |products|; the FP8
parity tolerance of the other tests is derived from this figure.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
from gpu_util import DEV, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _fp8_gemm(qa, qb):
    """C = deq(qa) @ deq(qb) through mfg_gemm(FP8 | PRECONVERTED) with unit tile scales."""
    M, K = qa.shape
    N = qb.shape[1]
    def pack(q, rows, cols):
        off = mfg.lib().mfg_fp8_scale_offset(rows, cols)
        tr, tc = -(-rows // 128), -(-cols // 128)
        buf = np.zeros(off + 4 * tr * tc, np.uint8)
        buf[: rows * cols] = q.reshape(-1)
        buf[off:] = np.ones(tr * tc, np.float32).view(np.uint8)
        return torch.from_numpy(buf).to(DEV)
    A, B = pack(qa, M, K), pack(qb, K, N)
    C = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    st = mfg.lib().mfg_gemm(M, N, K, A.data_ptr(), K, B.data_ptr(), N, C.data_ptr(), N, 1.0, 0.0,
                            mfg.MFG_FP8_E4M3 | mfg.MFG_IN_PRECONVERTED, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    return host(C)


def _code(v):
    return oracle.e4m3_encode(np.array([v], np.float64))[0]


def test_small_terms_next_to_large_ones_are_dropped():
    qa = np.zeros((32, 64), np.uint8)
    qb = np.zeros((64, 32), np.uint8)
    qa[0, 0], qa[0, 1] = _code(448.0), _code(2.0 ** -9)
    qb[0, 0], qb[1, 0] = _code(1.0), _code(1.0)
    qa[1, 0], qa[1, 1] = _code(1.0), _code(2.0 ** -9)       # same gap, smaller magnitude
    C = _fp8_gemm(qa, qb)
    assert C[0, 0] == 448.0                                  # exact FP32 sum would be 448.001953125
    assert C[1, 0] == 1.0 + 2.0 ** -9                        # kept: within the instruction's precision


def test_error_below_2_to_minus_12_of_abs_sum():
    rng = np.random.default_rng(0)
    codes = np.arange(256, dtype=np.uint8)
    finite = codes[np.isfinite(oracle.e4m3_decode(codes))]
    qa = rng.choice(finite, size=(128, 64)).astype(np.uint8)
    qb = rng.choice(finite, size=(64, 128)).astype(np.uint8)
    C = _fp8_gemm(qa, qb)
    a, b = oracle.e4m3_decode(qa), oracle.e4m3_decode(qb)
    exact = oracle.gemm(a, b)
    absum = oracle.gemm(np.abs(a), np.abs(b))
    rel = np.abs(C - exact) / np.maximum(absum, 1e-300)
    print(f"max |C - exact| / sum|p| = 2^{np.log2(rel.max()):.2f}")
    assert rel.max() <= 2.0 ** -11.75
