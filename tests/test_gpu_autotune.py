"""GPU tests of the autotuner (mfg_autotune): it times every configuration of a
mode, keeps the fastest one whose output is bitwise equal to configuration
0's, records it in the tuned table, and mfg_gemm then uses it -- with the
same bits and within the oracle's parity tolerance."""
import ctypes

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
    mfg.lib().mfg_tune_clear()
    yield
    mfg.lib().mfg_tune_clear()


@pytest.mark.parametrize("mode,shape,pre", [
    ("f16", (1024, 1024, 1024), True),
    ("bf16", (512, 768, 384), True),
    ("split3", (512, 384, 320), False),
    ("f32", (384, 256, 192), False),
])
def test_autotune_picks_a_bitwise_equal_config(mode, shape, pre):
    M, N, K = shape
    A, B = workloads.uniform(31, [(M, K), (K, N)])
    if pre:
        dt = torch.float16 if mode == "f16" else torch.bfloat16
        dA, dB = dev(A).to(dt), dev(B).to(dt)
    else:
        dA, dB = dev(A), dev(B)
    C = torch.empty((M, N), dtype=torch.float32, device=DEV)
    best, ms = mfg.autotune(dA, dB, C, mode, reps=2, preconverted=pre)
    assert 0 <= best < mfg.num_configs(mode) and ms > 0
    m = mfg.mode_of(mode) | (mfg.MFG_IN_PRECONVERTED if pre else 0)
    assert mfg.lib().mfg_tune_lookup(M, N, K, m) == best
    # the default path now runs the tuned configuration: same bits as configuration 0
    c_def = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    c_ref = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    mfg.gemm(dA, dB, c_def, 1.0, 0.0, mode=mode, preconverted=pre)
    mfg.gemm(dA, dB, c_ref, 1.0, 0.0, mode=mode, preconverted=pre, config=0)
    got = host(c_def)
    assert np.array_equal(got.view(np.uint32), host(c_ref).view(np.uint32))
    if pre:  # operands already rounded: the F32 reference of the rounded values
        ref = oracle.reference("f32", host(dA.float()), host(dB.float()))
    else:
        ref = oracle.reference(mode, A, B)
    assert_parity(got, ref, f"{mode} tuned config {best}", mode=mode)


def test_tuned_table_survives_save_and_load(tmp_path):
    M = N = K = 512
    A, B = workloads.uniform(32, [(M, K), (K, N)])
    dA, dB = dev(A).half(), dev(B).half()
    C = torch.empty((M, N), dtype=torch.float32, device=DEV)
    best, _ = mfg.autotune(dA, dB, C, "f16", reps=1, preconverted=True)
    path = str(tmp_path / "tuned.txt").encode()
    assert mfg.lib().mfg_tune_save(path) == 0
    mfg.lib().mfg_tune_clear()
    assert mfg.lib().mfg_tune_load(path) == 0
    assert mfg.lib().mfg_tune_lookup(M, N, K, mfg.MFG_F16) == best


def test_autotune_rejects_bad_arguments():
    C = torch.empty((8, 8), dtype=torch.float32, device=DEV)
    A = torch.empty((8, 8), dtype=torch.float16, device=DEV)
    with pytest.raises(mfg.MfgError):
        mfg.autotune(A, A, C, "f16", reps=0, preconverted=True)
    best = ctypes.c_int()
    st = mfg.lib().mfg_autotune(8, 8, 8, None, 8, A.data_ptr(), 8, C.data_ptr(), 8, mfg.MFG_F16 | mfg.MFG_IN_PRECONVERTED,
                                1, ctypes.byref(best), None, None)
    assert st == mfg.capi.MFG_ERR_INVALID_ARG


def test_tuned_config_that_does_not_serve_the_shape_falls_back(tmp_path):
    """The tuned table is keyed by power-of-two size buckets.  An entry naming
    a kernel that needs K % 64 == 0 and N % 8 == 0 (the 256 x 256 pipelined
    configuration) must not break a same-bucket shape without them: mfg_gemm
    falls back to the default choice, bitwise equal to configuration 0."""
    cfg = next(i for i in range(mfg.num_configs("f16")) if mfg.config_name("f16", i).startswith("q256x256"))
    path = tmp_path / "tuned.txt"
    path.write_text(f"{mfg.MFG_F16} 10 10 10 {cfg}\n")  # bucket of sizes 1024 .. 2047
    assert mfg.lib().mfg_tune_load(str(path).encode()) == 0
    assert mfg.lib().mfg_tune_lookup(1024, 1024, 1024, mfg.MFG_F16) == cfg
    M, N, K = 1100, 1036, 1030  # same bucket; K % 64 != 0, N % 8 != 0
    A, B = workloads.uniform(33, [(M, K), (K, N)])
    sa = torch.zeros((M, 1032), dtype=torch.float16, device=DEV)
    sb = torch.zeros((K, 1040), dtype=torch.float16, device=DEV)
    sa[:, :K] = dev(A).half()
    sb[:, :N] = dev(B).half()
    dA, dB = sa[:, :K], sb[:, :N]
    c = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    c0 = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    mfg.gemm(dA, dB, c, 1.0, 0.0, mode="f16", preconverted=True)
    mfg.gemm(dA, dB, c0, 1.0, 0.0, mode="f16", preconverted=True, config=0)
    assert np.array_equal(host(c).view(np.uint32), host(c0).view(np.uint32))
    for mode, m32 in (("split3", mfg.MFG_F16_SPLIT3), ("f16", mfg.MFG_F16)):  # library-converted operands too
        path.write_text(f"{m32} 10 10 10 {mfg.num_configs(mode) - 1}\n")
        mfg.lib().mfg_tune_clear()
        assert mfg.lib().mfg_tune_load(str(path).encode()) == 0
        c = torch.zeros((M, N), dtype=torch.float32, device=DEV)
        c0 = torch.zeros((M, N), dtype=torch.float32, device=DEV)
        mfg.gemm(dev(A), dev(B), c, 1.0, 0.0, mode=mode)
        mfg.gemm(dev(A), dev(B), c0, 1.0, 0.0, mode=mode, config=0)
        assert np.array_equal(host(c).view(np.uint32), host(c0).view(np.uint32)), mode
