"""Pins of the oracle's linear-solve references (the iterative-refinement
consumer of the GEMM; paper Sec. V cites the technique).

* lu_partial_pivot is checked against a different implementation (SciPy's
  LAPACK getrf through lu_factor) -- same pivots, same factors -- and by
  reconstruction P A = L U;
* its pivot rule on a matrix that needs a swap, and the first-maximum rule on
  ties, are fixed by hand;
* solve reproduces an integer system's exact rational solution (Gaussian
  elimination in Fractions);
* backward_error is checked on a hand-computed case and on a solution that
  is exact to rounding.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _lu_parts(LU):
    L = np.tril(LU, -1) + np.eye(LU.shape[0])
    return L, np.triu(LU)


@pytest.mark.parametrize("n", [1, 2, 7, 50])
def test_lu_matches_lapack_and_reconstructs(n):
    scipy_linalg = pytest.importorskip("scipy.linalg")
    A = np.random.default_rng(n).standard_normal((n, n))
    LU, piv = oracle.lu_partial_pivot(A)
    lu2, piv2 = scipy_linalg.lu_factor(A)
    assert np.array_equal(piv, piv2)
    assert np.allclose(LU, lu2, rtol=0, atol=1e-12 * n)
    L, U = _lu_parts(LU)
    assert np.allclose(oracle.apply_pivots(piv, A), L @ U, rtol=0, atol=1e-13 * n)
    assert np.all(np.abs(np.tril(LU, -1)) <= 1.0)


def test_pivot_rule_by_hand():
    LU, piv = oracle.lu_partial_pivot([[0.0, 1.0], [2.0, 3.0]])
    assert list(piv) == [1, 1]
    assert np.array_equal(LU, [[2.0, 3.0], [0.0, 1.0]])
    # equal magnitudes: the first (upper) row stays
    LU, piv = oracle.lu_partial_pivot([[1.0, 2.0], [-1.0, 4.0]])
    assert list(piv) == [0, 1] and np.array_equal(LU, [[1.0, 2.0], [-1.0, 6.0]])


def _exact_solve(A, b):
    """Gauss-Jordan elimination in Fractions."""
    n = len(A)
    M = [[Fraction(x) for x in row] + [Fraction(y)] for row, y in zip(A, b)]
    for k in range(n):
        p = next(i for i in range(k, n) if M[i][k] != 0)
        M[k], M[p] = M[p], M[k]
        for i in range(n):
            if i != k and M[i][k] != 0:
                f = M[i][k] / M[k][k]
                M[i] = [a - f * c for a, c in zip(M[i], M[k])]
    return [M[i][n] / M[i][i] for i in range(n)]


def test_solve_matches_exact_rational_solution():
    A = [[4, -2, 1, 3], [3, 6, -4, 2], [2, 1, 8, -5], [1, -3, 2, 7]]
    b = [1, -2, 3, 4]
    x = oracle.solve(np.array(A, float), np.array(b, float))
    want = _exact_solve(A, b)
    for xi, wi in zip(x, want):
        assert abs(Fraction(float(xi)) - wi) <= Fraction(1, 10 ** 14) * max(1, abs(wi))


def test_backward_error_by_hand_and_at_rounding_level():
    # r = b - A x = (0, -2): 2 / (|A| 4 * |x| 1.5 + |b| 4) = 0.2
    assert oracle.backward_error([[2.0, 0.0], [0.0, 4.0]], [1.0, 1.5], [2.0, 4.0]) == pytest.approx(0.2, rel=0, abs=0)
    n = 200
    A = np.random.default_rng(9).standard_normal((n, n))
    B = np.random.default_rng(10).standard_normal((n, 3))
    assert oracle.backward_error(A, oracle.solve(A, B), B) <= n * 2.0 ** -52
    # a planted error in one entry is seen
    X = oracle.solve(A, B)
    X[5, 1] += 1e-4 * np.max(np.abs(X))
    assert oracle.backward_error(A, X, B) > 1e-8
