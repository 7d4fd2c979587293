"""Helpers for the GPU tests: move seeded inputs to the device, run a mode
through the C ABI, compare with the oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg

DEV = "cuda:0"

# oracle mode names <-> library modes
MODES = ["f32", "f16", "bf16", "refine_a", "split3", "split4", "fp8", "bf16_split3", "bf16_split6"]


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def run_gemm(mode, A, B, C0=None, alpha=1.0, beta=0.0, config=-1):
    """C = alpha*A*B + beta*C0 on the GPU with FP32 operands converted by the library."""
    M, N = A.shape[0], B.shape[1]
    dA, dB = dev(A), dev(B)
    dC = dev(C0.astype(np.float32)) if C0 is not None else torch.zeros((M, N), dtype=torch.float32, device=DEV)
    mfg.gemm(dA, dB, dC, alpha, beta, mode=mode, config=config)
    return host(dC)


# The gfx950 E4M3 matrix instruction does not add its 64 products exactly in
# FP32: measured, its error is at most 2^-12 of the sum of |products| of one
# instruction (tests/test_gpu_fp8_model.py pins this).  Summed over the
# instructions of a dot product that is <= 2^-12 * (|A~||B~|)_ij; the FP8
# parity bar takes twice that on top of the FP32 accumulation term.
FP8_MFMA_REL = 2.0 ** -11


def parity_tolerance(ref: oracle.Reference, mode: str = "") -> float:
    tol = oracle.parity_tol(ref)
    if mode == "bf16_split6" and ref.absval.size:
        # one FP32 accumulator over the six products: K' = 6 * (K rounded up to 64)
        kk = 6 * (-(-ref.K // 64) * 64)
        tol = 4.0 * (kk + 2) * 2.0 ** -24 * float(np.max(ref.absval))
    if mode == "fp8" and ref.absval.size:
        tol += FP8_MFMA_REL * float(np.max(ref.absval))
    return tol


def assert_parity(C, ref: oracle.Reference, what="", mode=""):
    tol = parity_tolerance(ref, mode or what.split(" ")[0])
    err = float(np.max(np.abs(C.astype(np.float64) - ref.value))) if C.size else 0.0
    assert np.all(np.isfinite(C)), f"{what}: non-finite output"
    assert err <= tol, f"{what}: |C - R_mode|_max = {err:.3e} > tol {tol:.3e}"
    return err, tol
