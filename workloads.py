"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers (numpy PCG64 via ``default_rng``); it
holds none of the method's arithmetic -- no rounding to half precision, no
residual split, no GEMM.  Both the FP64 oracle and the GPU path receive the
same arrays from here.

Workload recipes (all row-major, leading dimension = number of columns):

* paper precision study (Sec. VI / Sec. VII.B): entries uniform in [-1, 1],
  and uniform in [-16, 16] for the large-value example;
* refinement study: normal(0, 1), and sign * 2^u with u uniform in [-10, 10];
* batched study (Sec. IV.B, Sec. VI): many 16x16x16 problems, plus 64^3 and a
  grouped set whose M, N, K are log-uniform in [16, 512];
* serving: Poisson arrivals, sizes log-uniform in [32, 4096];
* linear solves: A = Q1 diag(s) Q2^T with Q1, Q2 the orthogonal factors of
  normal(0, 1) matrices and s log-spaced from 1 to the requested condition
  number (2-norm), right-hand sides normal(0, 1).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform(seed: int, shapes, lo: float = -1.0, hi: float = 1.0):
    """FP32 arrays with i.i.d. entries uniform in [lo, hi), drawn in order."""
    g = _rng(seed)
    return [g.uniform(lo, hi, size=s).astype(np.float32) for s in shapes]


def normal(seed: int, shapes):
    """FP32 arrays with i.i.d. standard-normal entries, drawn in order."""
    g = _rng(seed)
    return [g.standard_normal(size=s, dtype=np.float32) for s in shapes]


def pow2(seed: int, shapes, ulo: float = -10.0, uhi: float = 10.0):
    """FP32 arrays of sign * 2^u, u uniform in [ulo, uhi] (continuous), sign +-1."""
    g = _rng(seed)
    out = []
    for s in shapes:
        u = g.uniform(ulo, uhi, size=s)
        sign = np.where(g.random(size=s) < 0.5, -1.0, 1.0)
        out.append((sign * np.exp2(u)).astype(np.float32))
    return out


def small_ints(seed: int, shapes, lo: int = -8, hi: int = 8):
    """FP32 arrays of integers uniform in [lo, hi] (inclusive)."""
    g = _rng(seed)
    return [g.integers(lo, hi + 1, size=s).astype(np.float32) for s in shapes]


def by_name(dist: str, seed: int, shapes):
    if dist == "uniform":
        return uniform(seed, shapes)
    if dist == "uniform16":
        return uniform(seed, shapes, -16.0, 16.0)
    if dist == "normal":
        return normal(seed, shapes)
    if dist == "pow2":
        return pow2(seed, shapes)
    if dist == "ints":
        return small_ints(seed, shapes)
    raise ValueError(dist)


def loguniform_dims(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """(count, 3) int64 array of (M, N, K), each round(exp(U(ln lo, ln hi))) in [lo, hi]."""
    g = _rng(seed)
    v = np.exp(g.uniform(np.log(lo), np.log(hi), size=(count, 3)))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


def poisson_arrivals(seed: int, rate: float, n: int) -> np.ndarray:
    """Arrival times (seconds, increasing) of a Poisson process with the given rate."""
    g = _rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, size=n))


def serving_trace(seed: int, rate: float, n: int, lo: int = 32, hi: int = 4096,
                  modes=("f16", "bf16", "split3", "fp8")):
    """Requests of the serving study: arrival time, (M, N, K), mode, pool offsets.

    Operands are sub-blocks of resident 4096 x 4096 pools, so each request
    carries the row/column offset of its A block (rows, cols) and B block.
    """
    g = _rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    dims = np.clip(np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), size=(n, 3)))), lo, hi).astype(np.int64)
    mode_idx = g.integers(0, len(modes), size=n)
    reqs = []
    for i in range(n):
        M, N, K = (int(x) for x in dims[i])
        a_r = int(g.integers(0, hi - M + 1))
        a_c = int(g.integers(0, hi - K + 1))
        b_r = int(g.integers(0, hi - K + 1))
        b_c = int(g.integers(0, hi - N + 1))
        reqs.append({"t": float(t[i]), "M": M, "N": N, "K": K, "mode": modes[mode_idx[i]],
                     "a_off": (a_r, a_c), "b_off": (b_r, b_c)})
    return reqs


def conditioned(seed: int, n: int, cond: float) -> np.ndarray:
    """An n x n FP64 matrix of 2-norm condition number `cond`: Q1 diag(s) Q2^T,
    Q1 and Q2 orthogonal (QR of normal(0, 1) matrices), s log-spaced 1 .. cond."""
    g = _rng(seed)
    q1, _ = np.linalg.qr(g.standard_normal((n, n)))
    q2, _ = np.linalg.qr(g.standard_normal((n, n)))
    s = np.logspace(0.0, np.log10(cond), n) if n > 1 else np.ones(1)
    return (q1 * s) @ q2.T
