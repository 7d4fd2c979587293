"""Pins of the oracle's three-way bfloat16 split and its six-product GEMM.

The split applies the paper's residual definition (Sec. V, Eq. R) twice on
bfloat16 planes.  The pins here do not re-run the oracle's formulas:

* reconstruction: for FP32 x whose planes stay normal, h + r1 + r2 == x
  exactly (h keeps the top 8 significant bits, each residual is exact in
  FP32 and the next plane keeps its top 8 bits, which leaves at most 8 bits
  for r2); a plane that dropped or double-counted a difference breaks it;
* construction from known planes: x built as h + r1 + r2 from bfloat16
  values with separated exponents is split back into exactly those planes;
* the six-product sum on such inputs equals, in exact rational arithmetic,
  the six products of the constructed planes; and the exact product minus
  it equals the three dropped products r1 r2 + r2 r1 + r2 r2 exactly;
* on bfloat16-exact inputs the mode reduces to the plain bfloat16 GEMM.
"""
from fractions import Fraction

import numpy as np

import oracle


def _bf16_exact(v):
    return np.array_equal(oracle.bf16_round(v), np.asarray(v, dtype=np.float64))


def test_reconstruction_is_exact_over_wide_exponent_range():
    g = np.random.default_rng(11)
    e = g.integers(-100, 100, size=20000)
    x = (g.uniform(1.0, 2.0, size=e.size) * np.ldexp(1.0, e)).astype(np.float32)
    x[::2] *= -1
    sp = oracle.split3_bf16(x)
    x64 = x.astype(np.float64)
    assert np.array_equal(sp.h + sp.r1 + sp.r2, x64)
    for p in (sp.h, sp.r1, sp.r2):
        assert _bf16_exact(p)
    # each plane is at most half a bfloat16 ulp (2^-8 relative) of the one before
    assert np.all(np.abs(sp.r1) <= np.abs(sp.h) * 2.0 ** -8)
    assert np.all(np.abs(sp.r2) <= np.abs(sp.r1) * 2.0 ** -8)
    # the plane codes decode to the plane values
    for b, v in zip(sp.bits, (sp.h, sp.r1, sp.r2)):
        assert np.array_equal(oracle.bf16_decode(b), v)


def _planes(seed, shape):
    """h in +-(1, 2) on the bfloat16 grid (step 2^-7), r1 in +-(2^-9, 2^-8)
    (step 2^-16), r2 in +-[2^-18, 2^-17) (step 2^-23): x = h + r1 + r2 spans
    bits 2^0 .. 2^-23, so it is an FP32 value.  Keeping h and r1 one grid step
    inside their binades keeps x in h's binade and r1 + r2 in r1's, where
    |r1 + r2| < 2^-8 and |r2| < 2^-17 are below half a plane ulp, so each
    rounding lands on the constructed plane."""
    g = np.random.default_rng(seed)
    sgn = lambda: np.where(g.random(size=shape) < 0.5, -1.0, 1.0)
    h = sgn() * (1.0 + g.integers(1, 128, size=shape) * 2.0 ** -7)
    r1 = sgn() * (2.0 ** -9 + g.integers(1, 127, size=shape) * 2.0 ** -16)
    r2 = sgn() * (2.0 ** -18 + g.integers(0, 32, size=shape) * 2.0 ** -23)
    x = h + r1 + r2
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x)
    return x.astype(np.float32), h, r1, r2


def test_split_recovers_constructed_planes():
    x, h, r1, r2 = _planes(5, (64, 64))
    sp = oracle.split3_bf16(x)
    assert np.array_equal(sp.h, h)
    assert np.array_equal(sp.r1, r1)
    assert np.array_equal(sp.r2, r2)


def _fsum_products(P, Q, i, j):
    return sum(Fraction(float(P[i, k])) * Fraction(float(Q[k, j])) for k in range(P.shape[1]))


def test_six_products_and_dropped_terms_exact():
    M, K, N = 4, 7, 3
    A, ah, a1, a2 = _planes(21, (M, K))
    B, bh, b1, b2 = _planes(22, (K, N))
    ref = oracle.reference("bf16_split6", A, B).value
    ex = oracle.exact(A, B)
    kept = [(ah, bh), (ah, b1), (a1, bh), (ah, b2), (a1, b1), (a2, bh)]
    dropped = [(a1, b2), (a2, b1), (a2, b2)]
    for i in range(M):
        for j in range(N):
            want = sum(_fsum_products(P, Q, i, j) for P, Q in kept)
            assert Fraction(float(ref[i, j])) == want, (i, j)
            gone = sum(_fsum_products(P, Q, i, j) for P, Q in dropped)
            assert Fraction(float(ex[i, j])) - Fraction(float(ref[i, j])) == gone, (i, j)


def test_reduces_to_bf16_on_bf16_exact_inputs():
    g = np.random.default_rng(3)
    A = oracle.bf16_round(g.standard_normal((20, 33))).astype(np.float32)
    B = oracle.bf16_round(g.standard_normal((33, 9))).astype(np.float32)
    assert np.array_equal(oracle.reference("bf16_split6", A, B).value, oracle.reference("bf16", A, B).value)


def test_error_near_fp32_and_within_bound():
    g = np.random.default_rng(4)
    A = g.standard_normal((48, 256)).astype(np.float32)
    B = g.standard_normal((256, 40)).astype(np.float32)
    ex = oracle.exact(A, B)
    mag = oracle.gemm(np.abs(A), np.abs(B))
    err6 = np.abs(oracle.reference("bf16_split6", A, B).value - ex)
    err3 = np.abs(oracle.reference("bf16_split3", A, B).value - ex)
    # the dropped products are below 2^-23 |A||B| (|r1| <= 2^-8|a|, |r2| <= 2^-16|a|)
    assert np.all(err6 <= 2.0 ** -22 * mag)
    assert err6.max() < 2.0 ** -6 * err3.max()
    bnd = oracle.representation_bound("bf16_split6", A, B)
    assert np.all(err6 <= bnd * (1 + 1e-12) + 1e-300)
