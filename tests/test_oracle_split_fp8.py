"""Pins of the oracle's split-refinement and FP8 operands.

* Eq. R / Eq. 1 / Eq. 2 (paper Sec. V): with exact (unrounded) residuals the
  two- and four-product sums reproduce A_single B_half and A_single B_single;
  the scaled, FP16-rounded residual meets the 2^-22 representation bound;
  FP16-exact inputs give zero residuals, so every refined mode equals the
  plain FP16 mode.
* Each mode's distance to the exact product stays inside the a-priori bound,
  and mistakes (dropped product, wrong scale, wrong sign) fall outside it.
* FP8: power-of-two tile scales; integers |x| <= 16 are exact after scaling.
"""
import numpy as np
import pytest

import oracle
import workloads


def _binade_sweep(n=200_000, seed=0):
    rng = np.random.default_rng(seed)
    e = rng.uniform(-30, 15.9, n)
    x = (np.where(rng.random(n) < 0.5, -1, 1) * np.exp2(e)).astype(np.float32)
    return x


def test_residual_is_exact_and_head_plus_residual_is_x():
    x = _binade_sweep()
    sp = oracle.split_f16(x)
    r = x.astype(np.float64) - sp.head
    # the residual is exactly representable in FP32 (13 significant bits at most)
    assert np.array_equal(r.astype(np.float32).astype(np.float64), r)
    assert np.array_equal(sp.head + r, x.astype(np.float64))


def test_scaled_residual_representation_bound():
    x = _binade_sweep(seed=1)
    sp = oracle.split_f16(x)
    err = np.abs(x.astype(np.float64) - (sp.head + sp.resid / sp.s))
    assert np.all(err <= 2.0 ** -22 * np.abs(x.astype(np.float64)) + 2.0 ** -35)
    # without the residual the error is the FP16 rounding error, ~2^-11 relative
    err0 = np.abs(x.astype(np.float64) - sp.head)
    big = np.abs(x) > 2.0 ** -14
    assert np.max(err0[big] / np.abs(x[big])) > 2.0 ** -12


def test_fp16_exact_inputs_have_zero_residual():
    codes = np.arange(0, 0x7C00, dtype=np.uint32).astype(np.uint16)
    x = codes.view(np.float16).astype(np.float32)
    sp = oracle.split_f16(x)
    assert np.all(sp.resid == 0.0)
    assert np.array_equal(sp.head_bits, codes)


def test_eq1_and_eq2_identities_with_exact_residuals():
    A, B = workloads.normal(3, [(40, 64), (64, 24)])
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    Ah, Bh = oracle.f16_round(A), oracle.f16_round(B)
    RA, RB = A64 - Ah, B64 - Bh
    g = oracle.gemm
    scale = np.abs(A64) @ np.abs(B64)
    tol = 64 * 2.0 ** -50 * scale
    # Eq. 1: A_single B_half = R_A B_half + A_half B_half
    assert np.all(np.abs(g(RA, Bh) + g(Ah, Bh) - g(A64, Bh)) <= tol)
    # Eq. 2: A_single B_single = R_A R_B + A_half R_B + R_A B_half + A_half B_half
    four = g(RA, RB) + g(Ah, RB) + g(RA, Bh) + g(Ah, Bh)
    assert np.all(np.abs(four - g(A64, B64)) <= tol)


@pytest.mark.parametrize("mode", ["refine_a", "split3", "split4"])
def test_refined_modes_equal_f16_on_fp16_exact_inputs(mode):
    A, B = workloads.uniform(4, [(33, 48), (48, 17)])
    A = oracle.f16_round(A).astype(np.float32)
    B = oracle.f16_round(B).astype(np.float32)
    r16 = oracle.reference("f16", A, B).value
    rm = oracle.reference(mode, A, B).value
    assert np.array_equal(rm, r16)


@pytest.mark.parametrize("dist", ["uniform", "normal", "pow2"])
@pytest.mark.parametrize("mode", ["f16", "bf16", "refine_a", "split3", "split4", "fp8", "bf16_split3"])
def test_mode_reference_within_representation_bound(mode, dist):
    A, B = workloads.by_name(dist, 12, [(48, 160), (160, 40)])
    ex = oracle.exact(A, B)
    rm = oracle.reference(mode, A, B).value
    bnd = oracle.representation_bound(mode, A, B)
    slack = 64 * 2.0 ** -52 * (np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)))
    assert np.all(np.abs(rm - ex) <= bnd + slack)


def test_refinement_ordering_of_errors():
    A, B = workloads.uniform(13, [(64, 512), (512, 64)])
    ex = oracle.exact(A, B)
    err = {m: np.max(np.abs(oracle.reference(m, A, B).value - ex))
           for m in ("f16", "refine_a", "split3", "split4")}
    assert err["refine_a"] < err["f16"]
    assert err["split3"] < 2.0 ** -9 * err["f16"]   # ~2^-11 gain per operand
    assert err["split4"] <= err["split3"]
    # split3 and split4 differ by R_A R_B / s^2 only: <= 2^-22 |A||B| (to first order)
    d = np.abs(oracle.reference("split4", A, B).value - oracle.reference("split3", A, B).value)
    scale = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    assert np.all(d <= 2.0 ** -22 * (1 + 2.0 ** -9) * scale)


def _planted_split3(A, B, flavour):
    """A deliberately wrong SPLIT3 reference (mistakes planted on the CPU)."""
    sa, sb = oracle.split_f16(A), oracle.split_f16(B)
    g = oracle.gemm
    if flavour == "dropped":
        return g(sa.head, sb.head) + g(sa.head, sb.resid) / sa.s
    if flavour == "wrong_scale":
        return g(sa.head, sb.head) + (g(sa.head, sb.resid) + g(sa.resid, sb.head)) * sa.s
    if flavour == "wrong_sign":
        return g(sa.head, sb.head) - (g(sa.head, sb.resid) + g(sa.resid, sb.head)) / sa.s
    if flavour == "transposed":
        return g(sa.head, sb.head) + (g(sa.head, sb.resid) + g(sa.resid.T.copy(), sb.head)) / sa.s
    raise ValueError(flavour)


@pytest.mark.parametrize("flavour", ["dropped", "wrong_scale", "wrong_sign", "transposed"])
def test_bound_catches_planted_mistakes(flavour):
    A, B = workloads.normal(14, [(64, 64), (64, 64)])
    ex = oracle.exact(A, B)
    bnd = oracle.representation_bound("split3", A, B)
    bad = _planted_split3(A, B, flavour)
    assert np.any(np.abs(bad - ex) > bnd * 4)


def test_fp8_scale_exponents():
    f = oracle.fp8_scale_exponent
    assert f(448.0) == 0
    assert f(448.0001) == 1
    assert f(224.0) == -1
    assert f(224.0001) == 0
    assert f(1.0) == -8          # 448 * 2^-8 = 1.75 >= 1 > 0.875
    assert f(0.0) == 0
    assert f(2.0 ** -149) == -127  # clamped to the E8M0 range


def test_fp8_integers_are_exact():
    A, B = workloads.small_ints(15, [(200, 300), (300, 150)], -16, 16)
    qa, qb = oracle.fp8_quantize(A), oracle.fp8_quantize(B)
    assert np.array_equal(qa.deq, A.astype(np.float64))
    assert np.array_equal(qb.deq, B.astype(np.float64))
    assert qa.exps.shape == (2, 3) and qb.exps.shape == (3, 2)
    assert np.array_equal(oracle.reference("fp8", A, B).value, oracle.exact(A, B))


def test_fp8_quantize_uses_each_tile_scale():
    (A,) = workloads.normal(16, [(256, 256)])
    A[:128, :128] *= 1000.0
    q = oracle.fp8_quantize(A)
    assert q.exps[0, 0] > q.exps[1, 1] + 8
    # every code is finite and within +-448 after decoding
    v = oracle.e4m3_decode(q.codes)
    assert np.all(np.isfinite(v)) and np.max(np.abs(v)) <= 448.0
    # relative error of normal-range values <= 2^-4
    d = np.abs(q.deq - A.astype(np.float64))
    big = np.abs(A.astype(np.float64)) >= 2.0 ** -6 * np.repeat(np.repeat(q.scales, 128, 0), 128, 1)
    assert np.all(d[big] <= 2.0 ** -4 * np.abs(A.astype(np.float64))[big])


# ------------------------------------------------------------- BF16 split
def test_bf16_split_residual_exact_and_16_bit_bound():
    """Head rnebf16(x) and residual rnebf16(x - head), unscaled: x - head is exact in
    FP32, and head + residual is within 2^-16 |x| (two 8-bit significands) while the
    residual stays a normal number (|x| >= 2^-110), up to FP32's largest binade --
    where the FP16 split overflows.  Below that the residual loses bits in the
    subnormals, as the unscaled FP16 residual does below 2^-3."""
    rng = np.random.default_rng(3)
    e = rng.uniform(-110, 127.9, 200_000)
    x = (np.where(rng.random(e.size) < 0.5, -1, 1) * np.exp2(e)).astype(np.float32)
    x = x[np.isfinite(x)]
    sp = oracle.split_bf16(x)
    x64 = x.astype(np.float64)
    r = x64 - sp.head
    assert np.array_equal(r.astype(np.float32).astype(np.float64), r)
    assert sp.s == 1.0
    err = np.abs(x64 - (sp.head + sp.resid))
    assert np.all(err <= 2.0 ** -16 * np.abs(x64))
    # without the residual: bfloat16 rounding alone, up to 2^-8 relative
    assert np.max(np.abs(r) / np.abs(x64)) > 2.0 ** -10
    # the FP16 split cannot hold these magnitudes at all
    big = np.float32(1e30)
    assert np.isinf(oracle.split_f16(np.array([big])).head[0])
    assert oracle.split_bf16(np.array([big])).head[0] + oracle.split_bf16(np.array([big])).resid[0] == \
        pytest.approx(1e30, rel=2.0 ** -16)


def test_bf16_split_is_exact_on_16_bit_values():
    """A value that is the sum of two bfloat16 numbers, the second below half an
    ulp of the first and within FP32's 24 bits of it, is head + residual exactly."""
    rng = np.random.default_rng(4)
    a = oracle.bf16_round(rng.uniform(1, 2, 5000) * np.exp2(rng.integers(-20, 20, 5000)))
    sign = np.where(rng.random(5000) < 0.5, -1.0, 1.0)
    b = oracle.bf16_round(a * sign * np.exp2(-rng.uniform(9.1, 15.5, 5000)))
    x = (a + b).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), a + b)  # fits FP32
    sp = oracle.split_bf16(x)
    assert np.array_equal(sp.head + sp.resid, a + b)


def test_bf16_split3_equals_bf16_on_bf16_exact_inputs_and_ordering():
    A, B = workloads.small_ints(15, [(40, 96), (96, 24)], -100, 100)
    assert np.array_equal(oracle.reference("bf16_split3", A, B).value, oracle.reference("bf16", A, B).value)
    A, B = workloads.uniform(16, [(64, 512), (512, 64)])
    ex = oracle.exact(A, B)
    err = {m: np.max(np.abs(oracle.reference(m, A, B).value - ex)) for m in ("bf16", "bf16_split3", "split3")}
    assert err["bf16_split3"] < 2.0 ** -6 * err["bf16"]   # ~2^-8 gain per operand
    assert err["split3"] < err["bf16_split3"]             # 22 bits beat 16


@pytest.mark.parametrize("flavour", ["dropped", "scaled", "wrong_sign"])
def test_bf16_bound_catches_planted_mistakes(flavour):
    A, B = workloads.normal(17, [(64, 64), (64, 64)])
    ex = oracle.exact(A, B)
    bnd = oracle.representation_bound("bf16_split3", A, B)
    sa, sb = oracle.split_bf16(A), oracle.split_bf16(B)
    g = oracle.gemm
    if flavour == "dropped":
        bad = g(sa.head, sb.head) + g(sa.head, sb.resid)
    elif flavour == "scaled":  # the FP16 split's 2^-11 applied to unscaled residuals
        bad = g(sa.head, sb.head) + (g(sa.head, sb.resid) + g(sa.resid, sb.head)) / 2048.0
    else:
        bad = g(sa.head, sb.head) - (g(sa.head, sb.resid) + g(sa.resid, sb.head))
    assert np.any(np.abs(bad - ex) > bnd * 4)
