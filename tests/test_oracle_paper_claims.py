"""The oracle reproduces the precision figures the paper prints (Sec. VII.B).

The paper's error is ||e||_Max with e = C_half - C_single.  With exact FP64
accumulation the only error left is the input rounding of Sec. V, which is
what these tests measure (on sampled rows to keep the CPU suite short; the
max over a subset of rows can only be smaller than over all rows).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _claims():
    with open(os.path.join(GOLDEN, "paper_precision_claims.json")) as f:
        return json.load(f)


def _maxerr(mode, A, B, rows):
    ex = oracle.gemm(A, B, rows=rows)
    terms = oracle.mode_terms(mode, A, B)
    val = None
    for c, Ao, Bo in terms:
        g = c * oracle.gemm(Ao, Bo, rows=rows)
        val = g if val is None else val + g
    return float(np.max(np.abs(val - ex)))


@pytest.mark.slow
def test_uniform16_n4096_unrefined_error():
    """+-16 entries, N=4096: the paper measures ||e||_Max = 8.32 without refinement."""
    c = _claims()
    n = 4096
    A, B = workloads.uniform(5, [(n, n), (n, n)], -16.0, 16.0)
    rows = np.arange(0, n, 32)  # 128 rows
    e = _maxerr("f16", A, B, rows)
    assert 0.6 * c["uniform16_n4096_maxerr_unrefined"] < e < 1.3 * c["uniform16_n4096_maxerr_unrefined"]
    # two-sided refinement (Eq. 2): the paper reports 0.24 on its hardware, which
    # includes FP32 accumulation error; the input-rounding part alone is far smaller.
    e2 = _maxerr("split4", A, B, rows)
    assert e2 < c["uniform16_n4096_maxerr_eq2"]


def test_eq1_and_eq2_error_reduction_uniform():
    """Eq. 1 reduces the error by ~30% (A and B have equal norms); Eq. 2 by >= 10x."""
    c = _claims()
    n = 2048
    A, B = workloads.uniform(20, [(n, n), (n, n)])
    rows = np.arange(0, n, 16)
    e0 = _maxerr("f16", A, B, rows)
    e1 = _maxerr("refine_a", A, B, rows)
    e2 = _maxerr("split4", A, B, rows)
    expected_ratio = 1.0 - c["eq1_error_decrease_fraction_n8192"]
    assert abs(e1 / e0 - expected_ratio) < 0.12
    assert e0 / e2 >= c["eq2_error_decrease_factor_n8192"]


def test_error_grows_with_n():
    """The rounding error grows with N (per-entry work is K = N terms)."""
    errs = []
    ns = [256, 512, 1024, 2048]
    for n in ns:
        A, B = workloads.uniform(30 + n, [(n, n), (n, n)])
        rows = np.arange(0, n, max(1, n // 64))
        errs.append(_maxerr("f16", A, B, rows))
    slope = np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert all(b > a for a, b in zip(errs, errs[1:]))
    # random-sign rounding errors add up like sqrt(N): a slope near 1/2
    assert 0.3 < slope < 1.05
