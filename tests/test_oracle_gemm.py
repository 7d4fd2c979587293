"""Pins of the oracle's FP64 GEMM (paper Sec. IV: C = alpha*A*B + beta*C).

Closed forms (identity, permutation, all-ones), exact small-integer products
compared with Python's integer arithmetic, a pure-Python triple loop on tiny
random inputs, numpy's float64 matmul as an independent library routine, and
the BLAS edge conventions.
"""
import numpy as np
import pytest

import oracle
import workloads


def test_identity_gives_alpha_b_plus_beta_c():
    n = 37
    (B, C0) = workloads.uniform(1, [(n, 19), (n, 19)])
    I = np.eye(n)
    out = oracle.gemm(I, B, alpha=1.5, beta=-0.5, C0=C0)
    assert np.array_equal(out, 1.5 * B.astype(np.float64) - 0.5 * C0.astype(np.float64))


def test_permutation_permutes_rows():
    n = 29
    (B,) = workloads.uniform(2, [(n, 31)])
    perm = np.random.default_rng(0).permutation(n)
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    out = oracle.gemm(P, B)
    assert np.array_equal(out, B.astype(np.float64)[perm])


def test_all_ones_gives_k():
    M, N, K = 5, 7, 1000
    out = oracle.gemm(np.ones((M, K)), np.ones((K, N)))
    assert np.all(out == K)


def test_small_integers_exact_against_python_ints():
    A, B, C0 = workloads.small_ints(3, [(9, 40), (40, 11), (9, 11)])
    out = oracle.gemm(A, B, alpha=2.0, beta=-3.0, C0=C0)
    Ai, Bi, Ci = A.astype(int).tolist(), B.astype(int).tolist(), C0.astype(int).tolist()
    for i in range(9):
        for j in range(11):
            s = sum(Ai[i][k] * Bi[k][j] for k in range(40))
            assert out[i, j] == 2 * s - 3 * Ci[i][j]


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 2, 5), (7, 9, 4), (16, 17, 15)])
def test_brute_force_triple_loop(M, N, K):
    A, B, C0 = workloads.uniform(4, [(M, K), (K, N), (M, N)])
    out = oracle.gemm(A, B, alpha=0.75, beta=1.25, C0=C0)
    A64, B64, C64 = (x.astype(np.float64).tolist() for x in (A, B, C0))
    for i in range(M):
        for j in range(N):
            s = 0.0
            for k in range(K):
                s += A64[i][k] * B64[k][j]
            assert out[i, j] == 0.75 * s + 1.25 * C64[i][j]


def test_against_numpy_float64_matmul():
    A, B = workloads.normal(5, [(130, 257), (257, 66)])
    out = oracle.gemm(A, B)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    scale = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    assert np.all(np.abs(out - ref) <= 257 * 2.0 ** -52 * scale)


def test_row_subset_matches_full():
    A, B, C0 = workloads.uniform(6, [(64, 33), (33, 20), (64, 20)])
    full = oracle.gemm(A, B, 1.0, 1.0, C0)
    rows = np.array([0, 5, 31, 32, 63])
    assert np.array_equal(oracle.gemm(A, B, 1.0, 1.0, C0, rows=rows), full[rows])


def test_beta_zero_never_reads_c():
    A, B = workloads.uniform(7, [(8, 8), (8, 8)])
    C0 = np.full((8, 8), np.nan)
    out = oracle.gemm(A, B, 1.0, 0.0, C0)
    assert np.all(np.isfinite(out))


def test_k_zero_and_alpha_zero():
    (C0,) = workloads.uniform(8, [(4, 6)])
    out = oracle.gemm(np.zeros((4, 0)), np.zeros((0, 6)), 1.0, 2.0, C0)
    assert np.array_equal(out, 2.0 * C0.astype(np.float64))
    A, B = workloads.uniform(9, [(4, 5), (5, 6)])
    out = oracle.gemm(A, B, 0.0, 0.5, C0)
    assert np.array_equal(out, 0.5 * C0.astype(np.float64))


def test_exact_reference_matches_definition_rows():
    A, B, C0 = workloads.uniform(10, [(50, 70), (70, 30), (50, 30)])
    rows = oracle.sample_rows(50, n=10)
    r = oracle.exact(A, B, 1.0, 1.0, C0, rows=rows)
    assert np.array_equal(r, oracle.gemm(A, B, 1.0, 1.0, C0)[rows])


def test_parity_tol_formula():
    A, B = workloads.uniform(0, [(256, 256), (256, 256)])
    ref = oracle.reference("f16", A, B)
    tol = oracle.parity_tol(ref)
    # 4*(K+2)*2^-24*max(|A~||B~|): for uniform[-1,1] at K=256, max(|A||B|) is ~80
    assert tol == 4 * 258 * 2.0 ** -24 * float(np.max(ref.absval))
    assert 3e-3 < tol < 6e-3


def test_error_norms_closed_forms():
    # all-ones n x n error: max 1, Frobenius exactly n; a single spike sets the max norm
    n = 37
    ref = np.zeros((n, n))
    e = oracle.error_norms(np.ones((n, n), np.float32), ref)
    assert e["max_abs"] == 1.0 and e["fro"] == float(n) and e["ref_fro"] == 0.0 and e["ref_max"] == 0.0
    C = np.zeros((5, 4), np.float32)
    C[3, 2] = -2.5
    R = np.full((5, 4), 3.0)
    e = oracle.error_norms(C, R)
    assert e["max_abs"] == 5.5 and e["ref_max"] == 3.0 and e["ref_fro"] == np.sqrt(20 * 9.0)
    assert oracle.error_norms(np.zeros((0, 3)), np.zeros((0, 3)))["fro"] == 0.0


def test_sample_rows_cover_edges():
    rows = oracle.sample_rows(1000, n=40, seed=1)
    assert rows[0] == 0 and rows[-1] == 999 and len(rows) <= 40
    assert np.all(np.diff(rows) > 0)
