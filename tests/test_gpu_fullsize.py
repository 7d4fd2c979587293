"""Parity at the full problem size, in the launch configuration the benchmark times.

M = N = K = 8192 (the size the paper quotes its GEMM rates at, Sec. VI and
VII.A), inputs uniform in [-1, 1] from seed 2, C = A B + C (alpha = beta = 1),
every launch with the library's default configuration:

* F16 exactly as the benchmark's step runs it: the FP32 inputs rounded to FP16
  on the device (untimed there), then the GEMM on the preconverted operands;
* the refined modes (Sec. V, Eq. 1 and Eq. 2) and BF16 from the FP32 inputs,
  split by the library; at this size the two-plane kinds run on the 192 x 128
  tile, whose last tile row (rows 8064 .. 8191) is partial;
* FP8 from the FP32 inputs (128 x 128 tile quantisation on the device);
* M = N = K = 8000, partial tiles on both edges, in F16 and SPLIT3.

The oracle computes each mode's FP64 reference on sampled rows (first and last
rows, tile edges, rows of the partial last tile row, random rows), and every
element of those rows is compared with it to the same tolerance as the
small-size parity tests.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, assert_parity, dev, host, need_gpu

pytestmark = pytest.mark.gpu

N = 8192


@pytest.fixture(scope="module")
def inputs():
    need_gpu()
    A, B, C0 = workloads.uniform(2, [(N, N), (N, N), (N, N)])
    rows = np.union1d(oracle.sample_rows(N, n=16, seed=1), np.array([8064, 8127, 8128, 8190]))
    return A, B, C0, rows


def _check(mode, C, A, B, C0, rows):
    print(f"full-size parity: {mode}, N = {N}, {rows.size} sampled rows", flush=True)
    ref = oracle.reference(mode, A, B, 1.0, 1.0, C0, rows=rows)
    assert_parity(C[rows], ref, f"{mode} N={N}", mode)


def test_f16_headline_step(inputs):
    A, B, C0, rows = inputs
    dA32, dB32 = dev(A), dev(B)
    dA = torch.empty((N, N), dtype=torch.float16, device=DEV)
    dB = torch.empty((N, N), dtype=torch.float16, device=DEV)
    mfg.round_f16(dA32, dA)
    mfg.round_f16(dB32, dB)
    del dA32, dB32
    dC = dev(C0)
    mfg.gemm(dA, dB, dC, 1.0, 1.0, mode="f16", preconverted=True)
    _check("f16", host(dC), A, B, C0, rows)


@pytest.mark.parametrize("mode", ["split3", "refine_a", "bf16_split3", "bf16"])
def test_fp32_input_modes(inputs, mode):
    A, B, C0, rows = inputs
    dA, dB, dC = dev(A), dev(B), dev(C0)
    mfg.gemm(dA, dB, dC, 1.0, 1.0, mode=mode)
    _check(mode, host(dC), A, B, C0, rows)


def test_fp8_from_fp32(inputs):
    """FP8 from the FP32 inputs (tile quantisation on the device, the scaled
    FP8 GEMM): the oracle quantises B and the 128-row tile rows of A that hold
    the sampled rows (tiles are independent, so these equal the full
    quantisation's), and the sampled rows are compared at the FP8 bar."""
    A, B, C0, rows = inputs
    dA, dB, dC = dev(A), dev(B), dev(C0)
    mfg.gemm(dA, dB, dC, 1.0, 1.0, mode="fp8")
    C = host(dC)
    T = oracle.FP8_TILE
    tiles = {}
    for r in rows:
        t = int(r) // T
        if t not in tiles:
            tiles[t] = oracle.fp8_quantize(A[t * T:(t + 1) * T]).deq
    arows = np.stack([tiles[int(r) // T][int(r) % T] for r in rows])
    bq = oracle.fp8_quantize(B).deq
    print(f"full-size parity: fp8, N = {N}, {rows.size} sampled rows", flush=True)
    ref = oracle.reference("fp8", arows, bq, 1.0, 1.0, C0[rows], terms=[(1.0, arows, bq)])
    assert_parity(C[rows], ref, f"fp8 N={N}", "fp8")


NR = 8000  # a multiple of 64 but not of the tiles: partial edge tiles at full scale


@pytest.mark.parametrize("mode", ["f16", "split3"])
def test_ragged_edges_at_scale(mode):
    """M = N = K = 8000: the pipelined kernels (K a multiple of 64) with
    partial tiles on the M and N edges (the last 256-row tile row holds 64
    rows, the last 192-row one of the split kinds 128), alpha = 1.25,
    beta = -0.5; rows from both edges and the tile boundaries before them."""
    need_gpu()
    A, B, C0 = workloads.uniform(3, [(NR, NR), (NR, NR), (NR, NR)])
    rows = np.union1d(oracle.sample_rows(NR, n=12, seed=4), np.array([7679, 7680, 7871, 7872, 7935, 7936, 7999]))
    dA, dB, dC = dev(A), dev(B), dev(C0)
    mfg.gemm(dA, dB, dC, 1.25, -0.5, mode=mode)
    C = host(dC)
    print(f"ragged parity: {mode}, N = {NR}, {rows.size} sampled rows", flush=True)
    ref = oracle.reference(mode, A, B, 1.25, -0.5, C0, rows=rows)
    assert_parity(C[rows], ref, f"{mode} N={NR}", mode)
