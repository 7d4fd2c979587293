"""The three-way bfloat16 split mode (MFG_BF16_SPLIT6) on the GPU.

Its conversion writes the planes h, r1, r2 of A and B (the paper's Eq. R
applied twice, bfloat16 planes) into one long-K operand pair, and a BF16 GEMM
over K' = 6 * (K rounded up to 64) sums the six products in one FP32
accumulator.  Parity is against the oracle's six-product reference within
the FP32-accumulation bar over K' terms; results are the same on every
configuration; the paths without a preconverted form report it.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, assert_parity, dev, host, need_gpu, run_gemm

pytestmark = pytest.mark.gpu
MODE = "bf16_split6"


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("shape", [(1, 1, 1), (33, 17, 5), (64, 64, 64), (130, 96, 65), (257, 190, 300),
                                   (512, 512, 1024), (96, 40, 2000)])
def test_parity_ragged_and_alpha_beta(shape):
    M, N, K = shape
    A, B, C0 = workloads.normal(41, [(M, K), (K, N), (M, N)])
    C = run_gemm(MODE, A, B, C0, 1.25, -0.5)
    ref = oracle.reference(MODE, A, B, 1.25, -0.5, C0)
    _, tol = assert_parity(C, ref, f"{MODE} {shape}", mode=MODE)
    # a-priori accuracy against the exact product
    bound = oracle.representation_bound(MODE, A, B, 1.25)
    assert np.all(np.abs(C - oracle.exact(A, B, 1.25, -0.5, C0)) <= bound + tol)


def test_every_config_bitwise_equal():
    M, N, K = 256, 264, 192
    A, B = workloads.uniform(42, [(M, K), (K, N)])
    ref = oracle.reference(MODE, A, B)
    outs = []
    for cfg in range(mfg.num_configs(MODE)):
        try:
            C = run_gemm(MODE, A, B, config=cfg)
        except mfg.MfgError as e:
            assert e.status == mfg.capi.MFG_ERR_UNSUPPORTED, mfg.config_name(MODE, cfg)
            continue
        assert_parity(C, ref, f"{MODE} cfg {cfg}", mode=MODE)
        outs.append(C)
    assert len(outs) >= 2
    for C in outs[1:]:
        assert np.array_equal(C.view(np.uint32), outs[0].view(np.uint32))


def test_full_fp32_range_planes_and_small_first_order():
    """sign * 2^u inputs over u in [-60, 60]: the planes stay normal, so the
    result matches the six-product reference at the FP32-accumulation bar
    relative to |A||B| even where plain BF16 loses 2^-8."""
    M, N, K = 96, 80, 256
    g = np.random.default_rng(43)
    A = (np.where(g.random((M, K)) < 0.5, -1, 1) * np.ldexp(g.uniform(1, 2, (M, K)), g.integers(-60, 60, (M, K))))
    B = (np.where(g.random((K, N)) < 0.5, -1, 1) * np.ldexp(g.uniform(1, 2, (K, N)), g.integers(-60, 60, (K, N))))
    A, B = A.astype(np.float32), B.astype(np.float32)
    C = run_gemm(MODE, A, B)
    assert_parity(C, oracle.reference(MODE, A, B), f"{MODE} wide range", mode=MODE)


def test_paths_without_a_preconverted_form_report_unsupported():
    L = mfg.lib()
    A, B = workloads.uniform(44, [(32, 32), (32, 32)])
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((32, 32), dtype=torch.float32, device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    m = mfg.capi.MFG_BF16_SPLIT6
    assert L.mfg_gemm(32, 32, 32, dA.data_ptr(), 32, dB.data_ptr(), 32, dC.data_ptr(), 32, 1.0, 0.0,
                      m | mfg.capi.MFG_IN_PRECONVERTED, s) == mfg.capi.MFG_ERR_UNSUPPORTED
    assert L.mfg_convert(32, 32, dA.data_ptr(), 32, dC.data_ptr(), 32, m, s) == mfg.capi.MFG_ERR_UNSUPPORTED
    with pytest.raises(mfg.MfgError) as e:
        mfg.gemm_batched(dA.view(1, 32, 32), dB.view(1, 32, 32), dC.view(1, 32, 32), mode=MODE)
    assert e.value.status == mfg.capi.MFG_ERR_UNSUPPORTED
    with pytest.raises(mfg.MfgError) as e:
        mfg.GroupedPlan([(dA, dB, dC)], mode=MODE)
    assert e.value.status == mfg.capi.MFG_ERR_UNSUPPORTED
    assert np.all(host(dC) == 0)
