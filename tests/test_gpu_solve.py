"""The iterative-refinement solver built on the GEMM (mfg_lu_factor,
mfg_lu_solve, mfg_solve_ir) against the oracle's FP64 references.

* LU: P A = L U to FP32 accuracy, |L| <= 1, a valid pivot sequence; on
  matrices whose pivots are unambiguous, the same pivots as the oracle's
  elimination (elsewhere FP32 rounding may break near-ties differently --
  both are correct partial-pivoting factorisations).
* solve with the factors: within FP32 accuracy times the condition number.
* refinement: for each factorisation mode, the backward error of the result
  reaches the FP64 level (below the tolerance) and the solution matches the
  oracle's FP64 solve within cond * tol; exactly singular matrices report
  the zero pivot.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, dev, host, need_gpu

pytestmark = pytest.mark.gpu
TOL = 2.0 ** -50


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _lu_parts(LU):
    L = np.tril(LU, -1) + np.eye(LU.shape[0])
    return L, np.triu(LU)


@pytest.mark.parametrize("n", [1, 5, 64, 65, 200, 513])
@pytest.mark.parametrize("mode", ["f32", "split3"])
def test_lu_factor_reconstructs(n, mode):
    A = workloads.normal(800 + n, [(n, n)])[0]
    dA = dev(A)
    ipiv, info = mfg.lu_factor(dA, mode)
    assert info == 0
    LU, piv = host(dA).astype(np.float64), host(ipiv).astype(np.int64)
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    L, U = _lu_parts(LU)
    assert np.all(np.abs(np.tril(LU, -1)) <= 1.0)
    err = np.max(np.abs(oracle.apply_pivots(piv, A) - L @ U))
    scale = np.max(np.abs(L) @ np.abs(U))
    assert err <= 4 * n * 2.0 ** -24 * scale, (err, scale)


def test_lu_pivots_match_oracle_when_unambiguous():
    """Each column's largest candidate beats the runner-up by far: integers
    with a dominant entry placed off the diagonal."""
    n = 150
    g = np.random.default_rng(5)
    A = g.integers(-3, 4, size=(n, n)).astype(np.float64)
    perm = g.permutation(n)
    A[perm, np.arange(n)] = 1000.0 + np.arange(n)  # column k: one dominant row
    dA = dev(A.astype(np.float32))
    ipiv, info = mfg.lu_factor(dA, "f32")
    _, piv = oracle.lu_partial_pivot(A)
    assert info == 0 and np.array_equal(host(ipiv).astype(np.int64), piv)


def test_lu_pivot_takes_first_of_equal_maxima_and_skips_nan():
    """Column 0 holds |5| at rows 1042, 530, 1030, 700 (530 and 1042 in one
    thread's registers, 1030 in another thread of its wavefront, 700 in another
    wavefront) and a NaN at row 20: the pivot is row 530, the first of the
    largest (the oracle's argmax rule), and the NaN is never taken."""
    n = 1100
    A = 0.1 * workloads.normal(81, [(n, n)])[0]
    A[[1042, 530, 1030, 700], 0] = [5.0, -5.0, 5.0, -5.0]
    A[20, 0] = np.nan
    ipiv, _ = mfg.lu_factor(dev(A), "f32")
    assert int(host(ipiv)[0]) == 530


# (70, 65539): more right-hand sides than a grid dimension holds, solved block by block
@pytest.mark.parametrize("n,nrhs", [(1, 1), (64, 3), (130, 1), (500, 2), (70, 65539)])
def test_lu_solve_fp32_accuracy(n, nrhs):
    A = workloads.conditioned(900 + n, n, 100.0)
    B = workloads.normal(901 + n, [(n, nrhs)])[0].astype(np.float64)
    dA = dev(A.astype(np.float32))
    ipiv, info = mfg.lu_factor(dA, "f32")
    dB = dev(B.astype(np.float32))
    mfg.lu_solve(dA, ipiv, dB)
    X = host(dB).astype(np.float64)
    ref = oracle.solve(A, B)
    assert np.max(np.abs(X - ref)) <= 100.0 * n * 2.0 ** -24 * 10 * np.max(np.abs(ref))


@pytest.mark.parametrize("mode,cond,max_iter", [("f32", 1e4, 10), ("split3", 1e4, 10), ("bf16_split3", 1e3, 12),
                                                ("f16", 10.0, 40), ("bf16", 10.0, 60)])
@pytest.mark.parametrize("n", [100, 257, 1024])
def test_solve_ir_reaches_fp64(mode, cond, max_iter, n):
    A = workloads.conditioned(1000 + n, n, cond)
    B = workloads.normal(1001 + n, [(n, 2)])[0].astype(np.float64)
    dX = torch.zeros((n, 2), dtype=torch.float64, device=DEV)
    r = mfg.solve_ir(dev(A), dev(B), dX, mode=mode, max_iter=max_iter, tol=TOL)
    X = host(dX)
    assert r["info"] == 0 and r["berr"] <= TOL, (mode, n, r)
    # the library's backward error is the oracle's
    be = oracle.backward_error(A, X, B)
    assert be <= 2 * TOL
    # forward error: within the infinity-norm condition number times the
    # backward errors of both solutions
    ref = oracle.solve(A, B)
    kinf = np.max(np.sum(np.abs(A), axis=1)) * np.max(np.sum(np.abs(np.linalg.inv(A)), axis=1))
    assert np.max(np.abs(X - ref)) <= 4 * kinf * (TOL + oracle.backward_error(A, ref, B)) * np.max(np.abs(ref))
    print(mode, n, r)


def test_solve_ir_large_on_refined_products():
    """n = 4096, the trailing updates (most of the flops) on the SPLIT3 matrix-core path."""
    n = 4096
    A = workloads.conditioned(77, n, 1e3)
    B = workloads.normal(78, [(n, 1)])[0].astype(np.float64)
    dX = torch.zeros((n, 1), dtype=torch.float64, device=DEV)
    r = mfg.solve_ir(dev(A), dev(B), dX, mode="split3", max_iter=10, tol=TOL)
    assert r["info"] == 0 and r["berr"] <= TOL and r["iters"] <= 6, r
    X = host(dX)
    assert oracle.backward_error(A, X, B) <= 2 * TOL


def test_solve_ir_tall_first_panel():
    """n = 8200: the first panel has more rows than the register-resident
    sub-panel kernel holds (8192) and is factored column by column in global
    memory; the later panels take the sub-panel path."""
    n = 8200
    A = workloads.normal(79, [(n, n)])[0].astype(np.float64)
    B = workloads.normal(80, [(n, 1)])[0].astype(np.float64)
    dX = torch.zeros((n, 1), dtype=torch.float64, device=DEV)
    r = mfg.solve_ir(dev(A), dev(B), dX, mode="f32", max_iter=10, tol=TOL)
    assert r["info"] == 0 and r["berr"] <= TOL, r
    assert oracle.backward_error(A, host(dX), B) <= 2 * TOL


def test_singular_and_empty():
    n = 70
    A = workloads.normal(5, [(n, n)])[0].astype(np.float64)
    A[:, 17] = 0.0  # column 17 exactly zero: the pivot of step 17 is zero
    B = np.ones((n, 1))
    dX = torch.full((n, 1), 7.0, dtype=torch.float64, device=DEV)
    r = mfg.solve_ir(dev(A), dev(B), dX, mode="f32")
    assert r["info"] == 18 and bool(torch.all(dX == 7.0))
    dA = dev(A.astype(np.float32))
    _, info = mfg.lu_factor(dA, "f32")
    assert info == 18
    # empty systems: nothing to do
    e = torch.zeros((0, 0), dtype=torch.float64, device=DEV)
    assert mfg.solve_ir(e, torch.zeros((0, 1), dtype=torch.float64, device=DEV),
                        torch.zeros((0, 1), dtype=torch.float64, device=DEV))["iters"] == 0


def test_invalid_arguments():
    L = mfg.lib()
    dA = torch.zeros((4, 4), dtype=torch.float32, device=DEV)
    ipiv = torch.zeros(4, dtype=torch.int32, device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    assert L.mfg_lu_factor(4, dA.data_ptr(), 3, ipiv.data_ptr(), None, mfg.capi.MFG_F32, s) == \
        mfg.capi.MFG_ERR_INVALID_ARG  # lda < n
    assert L.mfg_lu_factor(4, dA.data_ptr(), 4, ipiv.data_ptr(), None, mfg.capi.MFG_F32 | 0x100, s) == \
        mfg.capi.MFG_ERR_INVALID_ARG  # flags
    assert L.mfg_lu_factor(-1, dA.data_ptr(), 4, ipiv.data_ptr(), None, mfg.capi.MFG_F32, s) == \
        mfg.capi.MFG_ERR_INVALID_ARG
