"""Pins of the oracle's alpha / beta path (paper Sec. IV: C = alpha*A*B + beta*C).

Every mode's reference is checked at alpha not in {0, 1} and beta != 0
against exact rational arithmetic (Python ``Fraction``) on inputs built so
that each mode's operand form is known in closed form:

* small integers are exact in every 16-bit format and in E4M3 with a
  power-of-two tile scale, so every mode reduces to the integer product;
* a = H + R * 2^-11 with H an integer in +-[9, 15] and R an integer in
  [-7, 7] lies in [8, 16) in magnitude, so it has FP16 head H
  (|R * 2^-11| < half an FP16 ulp there, 2^-8) and
  scaled residual exactly R, so Eq. 1 / Eq. 2 (Sec. V) have closed forms;
* a = H + R * 2^-8 likewise has bfloat16 head H and unscaled residual
  R * 2^-8.

Every value involved is a dyadic rational with few significant bits, so the
FP64 reference is exact whatever its summation order, and equality is the
bar.  A reference that applied alpha to beta*C0 too, applied it to one
term only, or dropped it (value or magnitude) fails here.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

ALPHA = 2.5
BETA = -0.75


def _ints(seed, shape, lo, hi):
    return np.random.default_rng(seed).integers(lo, hi + 1, size=shape)


def _heads(seed, shape):
    """Integers with magnitude in [9, 15] and a random sign."""
    g = np.random.default_rng(seed)
    mag = g.integers(9, 16, size=shape)
    return np.where(g.random(size=shape) < 0.5, -mag, mag)


def _exact(Aterms, Bterms, coefs, C0, alpha, beta):
    """alpha * sum_t coef_t * (A_t @ B_t) + beta * C0, as Fractions (host loops)."""
    M, K = len(Aterms[0]), len(Aterms[0][0])
    N = len(Bterms[0][0])
    out = [[None] * N for _ in range(M)]
    mag = [[None] * N for _ in range(M)]
    a_al, a_be = Fraction(alpha), Fraction(beta)
    for i in range(M):
        for j in range(N):
            v = Fraction(0)
            m = Fraction(0)
            for At, Bt, c in zip(Aterms, Bterms, coefs):
                s = sum(Fraction(At[i][k]) * Fraction(Bt[k][j]) for k in range(K))
                sa = sum(abs(Fraction(At[i][k])) * abs(Fraction(Bt[k][j])) for k in range(K))
                v += c * s
                m += abs(c) * sa
            c0 = Fraction(float(C0[i][j]))
            out[i][j] = a_al * v + a_be * c0
            mag[i][j] = abs(a_al) * m + abs(a_be) * abs(c0)
    return out, mag


def _check(ref, want, mag):
    M, N = ref.value.shape
    for i in range(M):
        for j in range(N):
            assert Fraction(float(ref.value[i, j])) == want[i][j], (i, j)
            assert Fraction(float(ref.absval[i, j])) == mag[i][j], (i, j)


@pytest.mark.parametrize("mode", ["f32", "f16", "bf16", "refine_a", "split3", "split4", "bf16_split3", "bf16_split6", "fp8"])
def test_small_integers_every_mode(mode):
    M, N, K = 6, 5, 37
    A = _ints(1, (M, K), -8, 8).astype(np.float32)
    B = _ints(2, (K, N), -8, 8).astype(np.float32)
    C0 = _ints(3, (M, N), -9, 9).astype(np.float32)
    ref = oracle.reference(mode, A, B, ALPHA, BETA, C0)
    Ai, Bi = A.astype(int).tolist(), B.astype(int).tolist()
    # integers: every representation is exact, residuals vanish; the
    # magnitude sums |coef| |A_t||B_t| over the mode's terms, whose residual
    # terms are zero here
    want, mag = _exact([Ai], [Bi], [Fraction(1)], C0, ALPHA, BETA)
    _check(ref, want, mag)


def _split_inputs(seed, shape, step):
    H = _heads(seed, shape)
    R = _ints(seed + 100, shape, -7, 7)
    X = (H + R * step).astype(np.float32)
    assert np.array_equal(X.astype(np.float64), H + R * step)  # exact in FP32
    return X, H, R


@pytest.mark.parametrize("mode", ["refine_a", "split3", "split4", "f16", "f32"])
@pytest.mark.parametrize("alpha,beta", [(ALPHA, BETA), (-3.0, 0.5)])
def test_fp16_split_closed_form(mode, alpha, beta):
    M, N, K = 5, 4, 23
    s = Fraction(2048)
    A, HA, RA = _split_inputs(10, (M, K), 2.0 ** -11)
    B, HB, RB = _split_inputs(20, (K, N), 2.0 ** -11)
    C0 = _ints(30, (M, N), -9, 9).astype(np.float32)
    ref = oracle.reference(mode, A, B, alpha, beta, C0)
    ha, ra, hb, rb = HA.tolist(), RA.tolist(), HB.tolist(), RB.tolist()
    if mode == "f32":
        fa = [[Fraction(float(x)) for x in r] for r in A.astype(np.float64).tolist()]
        fb = [[Fraction(float(x)) for x in r] for r in B.astype(np.float64).tolist()]
        want, mag = _exact([fa], [fb], [Fraction(1)], C0, alpha, beta)
    elif mode == "f16":
        want, mag = _exact([ha], [hb], [Fraction(1)], C0, alpha, beta)
    elif mode == "refine_a":   # Eq. 1: A_h B_h + R_A B_h / s, B rounded to its head
        want, mag = _exact([ha, ra], [hb, hb], [Fraction(1), 1 / s], C0, alpha, beta)
    elif mode == "split3":     # Eq. 2 without R_A R_B
        want, mag = _exact([ha, ha, ra], [hb, rb, hb], [Fraction(1), 1 / s, 1 / s], C0, alpha, beta)
    else:                      # Eq. 2 in full
        want, mag = _exact([ha, ha, ra, ra], [hb, rb, hb, rb], [Fraction(1), 1 / s, 1 / s, 1 / s / s],
                           C0, alpha, beta)
    _check(ref, want, mag)


def test_bf16_split_closed_form():
    M, N, K = 5, 6, 19
    A, HA, RA = _split_inputs(40, (M, K), 2.0 ** -8)
    B, HB, RB = _split_inputs(50, (K, N), 2.0 ** -8)
    C0 = _ints(60, (M, N), -9, 9).astype(np.float32)
    ref = oracle.reference("bf16_split3", A, B, ALPHA, BETA, C0)
    q = Fraction(1, 256)
    ra = [[x * q for x in r] for r in RA.tolist()]
    rb = [[x * q for x in r] for r in RB.tolist()]
    want, mag = _exact([HA.tolist(), HA.tolist(), ra], [HB.tolist(), rb, HB.tolist()],
                       [Fraction(1)] * 3, C0, ALPHA, BETA)
    _check(ref, want, mag)


def test_exact_at_general_alpha_beta_is_f32_reference():
    A = _ints(70, (4, 9), -8, 8).astype(np.float32) / 4
    B = _ints(71, (9, 3), -8, 8).astype(np.float32) / 8
    C0 = _ints(72, (4, 3), -8, 8).astype(np.float32)
    want, _ = _exact([[[Fraction(float(x)) for x in r] for r in A.tolist()]],
                     [[[Fraction(float(x)) for x in r] for r in B.tolist()]], [Fraction(1)], C0, ALPHA, BETA)
    got = oracle.exact(A, B, ALPHA, BETA, C0)
    for i in range(4):
        for j in range(3):
            assert Fraction(float(got[i, j])) == want[i][j]


@pytest.mark.parametrize("mode", ["f16", "bf16", "refine_a", "split3", "split4", "bf16_split3", "bf16_split6", "fp8"])
def test_representation_bound_scales_with_abs_alpha(mode):
    A, B = (np.random.default_rng(80 + k).standard_normal(size=s).astype(np.float32)
            for k, s in enumerate([(24, 40), (40, 16)]))
    b1 = oracle.representation_bound(mode, A, B, alpha=1.0)
    assert np.all(b1 >= 0) and np.any(b1 > 0)
    # multiplying by a power of two is exact, so the scaling is bitwise
    assert np.array_equal(oracle.representation_bound(mode, A, B, alpha=2.0), 2.0 * b1)
    assert np.array_equal(oracle.representation_bound(mode, A, B, alpha=-0.5), 0.5 * b1)
    assert np.array_equal(oracle.representation_bound(mode, A, B, alpha=0.0), 0.0 * b1)


def test_representation_bound_holds_at_general_alpha():
    # |alpha R_mode - alpha R_exact| <= bound(alpha): the distance scales with |alpha|
    A, B = (np.random.default_rng(90 + k).uniform(-1, 1, size=s).astype(np.float32)
            for k, s in enumerate([(32, 48), (48, 20)]))
    for mode in ("f16", "refine_a", "split3", "split4", "bf16_split3", "bf16_split6", "fp8"):
        for alpha in (-1.75, 3.0):
            d = np.abs(oracle.reference(mode, A, B, alpha).value - oracle.exact(A, B, alpha))
            bnd = oracle.representation_bound(mode, A, B, alpha=alpha)
            assert np.all(d <= bnd * (1 + 1e-12) + 1e-300), mode


def _planted_reference(A, B, alpha, beta, C0, flavour):
    """Wrong alpha handling, planted on the CPU, in the mode-faithful F16 reference."""
    g = oracle.gemm
    Ah, Bh = oracle.f16_round(A), oracle.f16_round(B)
    c0 = C0.astype(np.float64)
    if flavour == "alpha_on_c":
        return alpha * (g(Ah, Bh) + beta * c0)
    if flavour == "alpha_dropped":
        return g(Ah, Bh) + beta * c0
    if flavour == "alpha_squared":
        return alpha * alpha * g(Ah, Bh) + beta * c0
    raise ValueError(flavour)


@pytest.mark.parametrize("flavour", ["alpha_on_c", "alpha_dropped", "alpha_squared"])
def test_planted_alpha_mistakes_are_caught(flavour):
    M, N, K = 6, 5, 37
    A = _ints(1, (M, K), -8, 8).astype(np.float32)
    B = _ints(2, (K, N), -8, 8).astype(np.float32)
    C0 = _ints(3, (M, N), -9, 9).astype(np.float32)
    want, _ = _exact([A.astype(int).tolist()], [B.astype(int).tolist()], [Fraction(1)], C0, ALPHA, BETA)
    bad = _planted_reference(A, B, ALPHA, BETA, C0, flavour)
    assert any(Fraction(float(bad[i, j])) != want[i][j] for i in range(M) for j in range(N))
