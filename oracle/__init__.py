"""FP64 CPU oracle for the mixed-precision GEMM library.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no
code with the GPU library (``paper_1803_04014_amd``) and never imports it.

What it computes (all in FP64 on the host):

* ``exact``: the plain definition ``alpha*A*B + beta*C0`` of the GEMM the
  paper studies (Sec. IV, first paragraph), from the original FP32 values.
  It replaces the paper's single-precision reference ``C_single`` of the
  error metric in Sec. VI.
* ``reference(mode, ...)``: the mode-faithful result -- the same GEMM on
  exactly the operands a mode hands to the matrix units, decoded to FP64 by
  this package's own rounding rules.  Split modes follow the paper's
  residual definition (Sec. V, Eq. R) and its one- and two-sided refinement
  identities (Sec. V, Eq. 1 and Eq. 2), with the residual scaled by 2^11
  before it is rounded to half precision (reading: an unscaled residual
  underflows into FP16 subnormals for |a| < 2^-3).
* bounds: the kernel-parity tolerance and an a-priori bound on the
  distance of each mode from the exact product.
* linear solve: LU with partial pivoting written out, the FP64 solve and
  the normwise backward error, the references of the iterative-refinement
  solver built on the GEMM (the technique Sec. V cites).

The rounding rules and the FP64 GEMM live in ``oracle.c`` (built into
``liboracle.so``); everything here composes them.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

# Residual scale of the split modes: the residual A - A_half is at most half
# an FP16 ulp of A, i.e. <= 2^-11 |A| for normal A; multiplying by 2^11
# brings it back to the magnitude of A before rounding it to FP16.
S_RESID = 2.0 ** 11
FP8_TILE = 128
E4M3_MAX = 448.0

MODES = ("f32", "f16", "bf16", "refine_a", "split3", "split4", "fp8", "bf16_split3", "bf16_split6")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, no FMA contraction)."""
    import subprocess

    cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           SRC_PATH, "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        build()
    L = ctypes.CDLL(LIB_PATH)
    d, i64, u16, u8 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint16, ctypes.c_uint8
    P = ctypes.c_void_p
    L.orc_f16_encode.argtypes, L.orc_f16_encode.restype = [d], u16
    L.orc_f16_decode.argtypes, L.orc_f16_decode.restype = [u16], d
    L.orc_bf16_encode.argtypes, L.orc_bf16_encode.restype = [d], u16
    L.orc_bf16_decode.argtypes, L.orc_bf16_decode.restype = [u16], d
    L.orc_e4m3_encode_sat.argtypes, L.orc_e4m3_encode_sat.restype = [d], u8
    L.orc_e4m3_decode.argtypes, L.orc_e4m3_decode.restype = [u8], d
    for name in ("orc_f16_encode_array", "orc_f16_decode_array", "orc_bf16_encode_array",
                 "orc_bf16_decode_array", "orc_e4m3_encode_array", "orc_e4m3_decode_array"):
        getattr(L, name).argtypes = [P, i64, P]
        getattr(L, name).restype = None
    L.orc_gemm_f64.argtypes = [i64, i64, i64, P, i64, P, i64, d, d, P, i64, P, i64, P, i64]
    L.orc_gemm_f64.restype = None
    L.orc_num_threads.argtypes, L.orc_num_threads.restype = [], ctypes.c_int
    _lib = L
    return L


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Number formats (paper Sec. V: 1 sign, 5 exponent, 10 fraction bits; RNE)
# --------------------------------------------------------------------------
def _map(fn_name, x, in_dtype, out_dtype):
    x = np.ascontiguousarray(np.asarray(x, dtype=in_dtype))
    out = np.empty(x.shape, dtype=out_dtype)
    getattr(lib(), fn_name)(_ptr(x), x.size, _ptr(out))
    return out


def f16_encode(x):
    return _map("orc_f16_encode_array", x, np.float64, np.uint16)


def f16_decode(h):
    return _map("orc_f16_decode_array", h, np.uint16, np.float64)


def bf16_encode(x):
    return _map("orc_bf16_encode_array", x, np.float64, np.uint16)


def bf16_decode(h):
    return _map("orc_bf16_decode_array", h, np.uint16, np.float64)


def e4m3_encode(x):
    return _map("orc_e4m3_encode_array", x, np.float64, np.uint8)


def e4m3_decode(q):
    return _map("orc_e4m3_decode_array", q, np.uint8, np.float64)


def f16_round(x):
    return f16_decode(f16_encode(x))


def bf16_round(x):
    return bf16_decode(bf16_encode(x))


@dataclass
class Split:
    """Head/residual pair of the paper's Eq. R, residual scaled by ``s``."""
    head_bits: np.ndarray   # uint16 FP16 codes of rne16(x)
    resid_bits: np.ndarray  # uint16 FP16 codes of rne16(s * (x - head))
    head: np.ndarray        # FP64 value of the head
    resid: np.ndarray       # FP64 value of the scaled residual
    s: float


def split_f16(x, s: float = S_RESID) -> Split:
    """Eq. R: R = x - x_half (exact in FP32 and FP64), stored as rne16(s*R)."""
    x64 = np.asarray(x, dtype=np.float64)
    hb = f16_encode(x64)
    h = f16_decode(hb)
    r = x64 - h
    rb = f16_encode(s * r)
    return Split(hb, rb, h, f16_decode(rb), s)


def split_bf16(x) -> Split:
    """Eq. R on bfloat16 planes: head rnebf16(x), residual rnebf16(x - head), unscaled
    (bfloat16 has FP32's exponent range, so the residual needs no scaling to stay
    out of the subnormals); x - head is exact in FP32 and FP64."""
    x64 = np.asarray(x, dtype=np.float64)
    hb = bf16_encode(x64)
    h = bf16_decode(hb)
    rb = bf16_encode(x64 - h)
    return Split(hb, rb, h, bf16_decode(rb), 1.0)


@dataclass
class Split3Way:
    """Eq. R applied twice on bfloat16 planes: x = h + r1 + r2 (+ what r2 rounds away)."""
    h: np.ndarray   # FP64 value of rnebf16(x)
    r1: np.ndarray  # FP64 value of rnebf16(x - h)
    r2: np.ndarray  # FP64 value of rnebf16(x - h - r1)
    bits: tuple     # uint16 bfloat16 codes of (h, r1, r2)


def split3_bf16(x) -> Split3Way:
    """Three-way bfloat16 split: the residual of Eq. R is itself split by Eq. R.
    Both differences are exact in FP64 (and in FP32 for FP32 x), so for FP32 x
    whose planes stay normal, h + r1 + r2 == x: each plane carries the next 8
    significant bits."""
    x64 = np.asarray(x, dtype=np.float64)
    hb = bf16_encode(x64)
    h = bf16_decode(hb)
    ab = bf16_encode(x64 - h)
    a = bf16_decode(ab)
    bb = bf16_encode((x64 - h) - a)
    return Split3Way(h, a, bf16_decode(bb), (hb, ab, bb))


@dataclass
class Fp8Tiles:
    """Per-tile FP8-E4M3 quantisation of a matrix."""
    codes: np.ndarray      # uint8, same shape as the input
    exps: np.ndarray       # int32 exponent E of each tile scale 2^E, tile-major
    scales: np.ndarray     # float64 2^E
    deq: np.ndarray        # float64 codes * scale, the values the GEMM sees
    tile: int


def fp8_scale_exponent(amax: float) -> int:
    """Smallest E with 448 * 2^E >= amax, clamped to [-127, 127]; 0 for amax == 0.

    Reading of the per-tile FP32 scale: a power of two, so that dividing by it
    is exact and values already on the FP8 grid stay exact.
    """
    if amax == 0.0:
        return 0
    e = int(np.ceil(np.log2(amax / E4M3_MAX)))
    while E4M3_MAX * 2.0 ** e < amax:
        e += 1
    while E4M3_MAX * 2.0 ** (e - 1) >= amax:
        e -= 1
    return max(-127, min(127, e))


def fp8_quantize(x, tile: int = FP8_TILE) -> Fp8Tiles:
    """Quantise a 2-D FP32 matrix to E4M3 with one power-of-two scale per tile."""
    x64 = np.asarray(x, dtype=np.float64)
    R, C = x64.shape
    tr, tc = -(-R // tile), -(-C // tile)
    exps = np.zeros((tr, tc), dtype=np.int32)
    codes = np.zeros((R, C), dtype=np.uint8)
    deq = np.zeros((R, C), dtype=np.float64)
    for ti in range(tr):
        for tj in range(tc):
            blk = x64[ti * tile:(ti + 1) * tile, tj * tile:(tj + 1) * tile]
            amax = float(np.max(np.abs(blk))) if blk.size else 0.0
            e = fp8_scale_exponent(amax)
            exps[ti, tj] = e
            q = e4m3_encode(blk / 2.0 ** e)
            codes[ti * tile:(ti + 1) * tile, tj * tile:(tj + 1) * tile] = q
            deq[ti * tile:(ti + 1) * tile, tj * tile:(tj + 1) * tile] = e4m3_decode(q) * 2.0 ** e
    return Fp8Tiles(codes, exps, np.ldexp(1.0, exps), deq, tile)


# --------------------------------------------------------------------------
# FP64 GEMM (paper Sec. IV: C = alpha*A*B + beta*C)
# --------------------------------------------------------------------------
def gemm(A, B, alpha: float = 1.0, beta: float = 0.0, C0=None, rows=None) -> np.ndarray:
    """FP64 ``alpha*A@B + beta*C0`` on rows ``rows`` (all rows when None)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    B = np.ascontiguousarray(np.asarray(B, dtype=np.float64))
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    if rows is None:
        rows_arr, nrows = None, M
    else:
        rows_arr = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nrows = rows_arr.size
        assert nrows == 0 or (rows_arr.min() >= 0 and rows_arr.max() < M)
    out = np.empty((nrows, N), dtype=np.float64)
    if beta != 0.0:
        C0 = np.ascontiguousarray(np.asarray(C0, dtype=np.float64))
        assert C0.shape == (M, N)
        c0p = _ptr(C0)
    else:
        c0p = None
    if nrows == 0 or N == 0:
        return out
    lib().orc_gemm_f64(M, N, K, _ptr(A), K, _ptr(B), N, float(alpha), float(beta),
                       c0p, N, _ptr(out), N,
                       None if rows_arr is None else _ptr(rows_arr), nrows)
    return out


# --------------------------------------------------------------------------
# Mode-faithful operands
# --------------------------------------------------------------------------
def mode_terms(mode: str, A, B):
    """Return [(coef, A_op, B_op)] with  result = sum coef * A_op @ B_op.

    f32      : A B
    f16/bf16 : rne(A) rne(B)
    refine_a : Eq. 1 -- A_h B_h + (R_A/s) B_h, B not split
    split3   : Eq. 2 without the R_A R_B product -- A_h B_h + (A_h R_B + R_A B_h)/s
    split4   : Eq. 2 -- split3 + R_A R_B / s^2
    bf16_split3 : Eq. 2 without R_A R_B on bfloat16 head and unscaled residual planes
    bf16_split6 : three-way bfloat16 split of A and B (split3_bf16), every product of
                  combined order <= 2: h h + (h r1 + r1 h) + (h r2 + r1 r1 + r2 h)
    fp8      : per-tile dequantised codes, deq(A) deq(B)
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if mode == "f32":
        return [(1.0, A, B)]
    if mode == "f16":
        return [(1.0, f16_round(A), f16_round(B))]
    if mode == "bf16":
        return [(1.0, bf16_round(A), bf16_round(B))]
    if mode == "refine_a":
        sa = split_f16(A)
        bh = f16_round(B)
        return [(1.0, sa.head, bh), (1.0 / sa.s, sa.resid, bh)]
    if mode in ("split3", "split4"):
        sa, sb = split_f16(A), split_f16(B)
        t = [(1.0, sa.head, sb.head), (1.0 / sa.s, sa.head, sb.resid), (1.0 / sa.s, sa.resid, sb.head)]
        if mode == "split4":
            t.append((1.0 / (sa.s * sb.s), sa.resid, sb.resid))
        return t
    if mode == "bf16_split3":
        sa, sb = split_bf16(A), split_bf16(B)
        return [(1.0, sa.head, sb.head), (1.0, sa.head, sb.resid), (1.0, sa.resid, sb.head)]
    if mode == "bf16_split6":
        a, b = split3_bf16(A), split3_bf16(B)
        return [(1.0, a.h, b.h), (1.0, a.h, b.r1), (1.0, a.r1, b.h),
                (1.0, a.h, b.r2), (1.0, a.r1, b.r1), (1.0, a.r2, b.h)]
    if mode == "fp8":
        return [(1.0, fp8_quantize(A).deq, fp8_quantize(B).deq)]
    raise ValueError(f"unknown mode {mode!r}")


def _rows_of(X, rows):
    X = np.asarray(X, dtype=np.float64)
    return X if rows is None else X[np.asarray(rows, dtype=np.int64)]


@dataclass
class Reference:
    value: np.ndarray   # FP64 alpha*sum(coef*A_op@B_op) + beta*C0 on the selected rows
    absval: np.ndarray  # FP64 |alpha|*sum(|coef|*|A_op|@|B_op|) + |beta|*|C0|
    K: int


def reference(mode: str, A, B, alpha: float = 1.0, beta: float = 0.0, C0=None,
              rows=None, terms=None) -> Reference:
    """Mode-faithful FP64 reference and the matching |.| magnitude for tolerances."""
    terms = mode_terms(mode, A, B) if terms is None else terms
    K = np.asarray(A).shape[1]
    val = None
    mag = None
    for coef, Aop, Bop in terms:
        g = gemm(Aop, Bop, rows=rows)
        ga = gemm(np.abs(Aop), np.abs(Bop), rows=rows)
        val = coef * g if val is None else val + coef * g
        mag = abs(coef) * ga if mag is None else mag + abs(coef) * ga
    val = alpha * val
    mag = abs(alpha) * mag
    if beta != 0.0:
        c0 = _rows_of(C0, rows)
        val = val + beta * c0
        mag = mag + abs(beta) * np.abs(c0)
    return Reference(val, mag, K)


def exact(A, B, alpha: float = 1.0, beta: float = 0.0, C0=None, rows=None) -> np.ndarray:
    """The plain definition alpha*A@B + beta*C0 from the FP32 inputs, in FP64."""
    return reference("f32", A, B, alpha, beta, C0, rows).value


def parity_tol(ref: Reference) -> float:
    """Kernel-parity tolerance: 4*(K+2)*2^-24 * max(|alpha||A_op||B_op| + |beta||C0|).

    Extends the 256^3 acceptance rule 4*K*2^-24*(|A||B|)_max (FP32 accumulation
    of K exact products, plus the alpha/beta epilogue) to general alpha, beta.
    """
    if ref.absval.size == 0:
        return 0.0
    return 4.0 * (ref.K + 2) * 2.0 ** -24 * float(np.max(ref.absval))


def representation_bound(mode: str, A, B, alpha: float = 1.0, rows=None) -> np.ndarray:
    """Elementwise a-priori bound on |R_mode - R_exact| (FP64, selected rows).

    With x~ the value a mode represents for x (rne16(x), h + R/s, deq(x), ...)
    and d = x - x~:  |AB - A~B~| <= |dA||B| + |A~||dB|; SPLIT3 also drops
    R_A R_B / s^2, bounded by |R_A||R_B|/s^2.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if mode == "f32":
        n = A.shape[0] if rows is None else len(rows)
        return np.zeros((n, B.shape[1]))
    if mode in ("f16", "bf16", "fp8"):
        At = mode_terms(mode, A, B)[0][1]
        Bt = mode_terms(mode, A, B)[0][2]
        extra = None
    elif mode == "bf16_split6":
        a, b = split3_bf16(A), split3_bf16(B)
        At, Bt = a.h + a.r1 + a.r2, b.h + b.r1 + b.r2
        # dropped products of combined order 3 and 4
        dropped = (gemm(np.abs(a.r1), np.abs(b.r2), rows=rows) + gemm(np.abs(a.r2), np.abs(b.r1), rows=rows)
                   + gemm(np.abs(a.r2), np.abs(b.r2), rows=rows))
        dA, dB = np.abs(A - At), np.abs(B - Bt)
        bnd = gemm(dA, np.abs(B), rows=rows) + gemm(np.abs(At), dB, rows=rows) + dropped
        return abs(alpha) * bnd
    elif mode == "refine_a":
        sa = split_f16(A)
        At = sa.head + sa.resid / sa.s
        Bt = f16_round(B)
        extra = None
    else:
        sa, sb = (split_bf16(A), split_bf16(B)) if mode == "bf16_split3" else (split_f16(A), split_f16(B))
        At = sa.head + sa.resid / sa.s
        Bt = sb.head + sb.resid / sb.s
        extra = (np.abs(sa.resid) / sa.s, np.abs(sb.resid) / sb.s) if mode in ("split3", "bf16_split3") else None
    dA, dB = np.abs(A - At), np.abs(B - Bt)
    bnd = gemm(dA, np.abs(B), rows=rows) + gemm(np.abs(At), dB, rows=rows)
    if extra is not None:
        bnd = bnd + gemm(extra[0], extra[1], rows=rows)
    return abs(alpha) * bnd


# --------------------------------------------------------------------------
# Linear solve (the consumer of Sec. V's refinement: iterative refinement)
# --------------------------------------------------------------------------
def lu_partial_pivot(A):
    """Gaussian elimination with partial pivoting in FP64, written out: for each
    column k the row of largest |value| on or below the diagonal (the first on
    ties) is swapped into row k, the column below is divided by the pivot and
    the trailing matrix gets the rank-1 update.  Returns (LU, piv): L unit lower
    below the diagonal, U on and above it, piv[k] the row swapped with row k."""
    a = np.array(A, dtype=np.float64)
    n = a.shape[0]
    piv = np.zeros(n, dtype=np.int64)
    for k in range(n):
        p = k + int(np.argmax(np.abs(a[k:, k])))  # argmax returns the first maximum
        piv[k] = p
        if p != k:
            a[[k, p], :] = a[[p, k], :]
        if a[k, k] != 0.0:
            a[k + 1:, k] /= a[k, k]
            a[k + 1:, k + 1:] -= np.outer(a[k + 1:, k], a[k, k + 1:])
    return a, piv


def apply_pivots(piv, X):
    """P X for the sequential row swaps piv (row k with row piv[k], k = 0, 1, ...)."""
    x = np.array(X, dtype=np.float64, copy=True)
    for k, p in enumerate(piv):
        if p != k:
            x[[k, int(p)]] = x[[int(p), k]]
    return x


def solve(A, B):
    """The solution of A X = B in FP64 (LAPACK's LU solve through numpy)."""
    return np.linalg.solve(np.asarray(A, dtype=np.float64), np.asarray(B, dtype=np.float64))


def backward_error(A, X, B) -> float:
    """Normwise backward error of X: max over columns j of
    |b_j - A x_j|_inf / (|A|_inf |x_j|_inf + |b_j|_inf), in FP64."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(A.shape[0], -1)
    B = np.asarray(B, dtype=np.float64).reshape(A.shape[0], -1)
    R = B - A @ X
    anorm = np.max(np.sum(np.abs(A), axis=1)) if A.size else 0.0
    worst = 0.0
    for j in range(X.shape[1]):
        den = anorm * np.max(np.abs(X[:, j])) + np.max(np.abs(B[:, j]))
        num = np.max(np.abs(R[:, j]))
        worst = max(worst, num / den if den > 0 else (np.inf if num > 0 else 0.0))
    return float(worst)


def error_norms(C, Cref) -> dict:
    """The paper's max norm of e = C - C_ref (Sec. VI) plus Frobenius norms, in FP64."""
    e = np.asarray(C, dtype=np.float64) - np.asarray(Cref, dtype=np.float64)
    r = np.asarray(Cref, dtype=np.float64)
    if e.size == 0:
        return {"max_abs": 0.0, "fro": 0.0, "ref_fro": 0.0, "ref_max": 0.0}
    return {
        "max_abs": float(np.max(np.abs(e))),
        "fro": float(np.sqrt(np.sum(e * e))),
        "ref_fro": float(np.sqrt(np.sum(r * r))),
        "ref_max": float(np.max(np.abs(r))),
    }


def sample_rows(M: int, n: int = 64, seed: int = 0) -> np.ndarray:
    """Rows checked at full size: first/last, tile edges (multiples of 16/32/128/256
    and their neighbours) and random rows, sorted and unique."""
    cand = {0, M - 1}
    for t in (16, 32, 128, 256):
        for b in range(t, M, t * max(1, M // (t * 8))):
            cand.update({b - 1, b})
    rng = np.random.default_rng(seed)
    cand.update(rng.integers(0, M, size=n).tolist())
    arr = np.array(sorted(c for c in cand if 0 <= c < M), dtype=np.int64)
    if arr.size > n:
        keep = np.unique(np.concatenate([arr[:2], arr[-2:], rng.choice(arr, n - 4, replace=False)]))
        arr = keep
    return arr
