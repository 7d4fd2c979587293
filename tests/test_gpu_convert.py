"""GPU parity of operand preparation and FP64 reductions against the oracle.

Conversions are integer-valued (bit patterns), so the bar is bit-exactness.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, dev, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _probe_floats():
    """Every FP16 value, its FP32 neighbours, midpoints and their neighbours,
    both signs, plus random FP32 bit patterns (finite and not)."""
    codes = np.arange(0, 0x7C00, dtype=np.uint32).astype(np.uint16)
    vals = codes.view(np.float16).astype(np.float32)
    nxt = np.append(vals[1:], np.float32(65536.0))
    mids = ((vals.astype(np.float64) + nxt.astype(np.float64)) / 2).astype(np.float32)
    pts = [vals, mids]
    for b in (vals, mids):
        pts += [np.nextafter(b, np.float32(np.inf)), np.nextafter(b, np.float32(-np.inf))]
    rng = np.random.default_rng(0)
    rnd = rng.integers(0, 2 ** 32, size=1 << 21, dtype=np.uint64).astype(np.uint32).view(np.float32)
    p = np.concatenate(pts + [rnd]).astype(np.float32)
    p = np.concatenate([p, -p])
    p = p[: p.size - p.size % 1024]
    return p.reshape(-1, 1024)


def test_round_f16_bit_exact():
    X = _probe_floats()
    out = torch.empty(X.shape, dtype=torch.int16, device=DEV)
    mfg.round_f16(dev(X), out)
    got = host(out).view(np.uint16)
    ref = oracle.f16_encode(X.astype(np.float64))
    nan = np.isnan(X)
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.all((got[nan] & 0x7C00) == 0x7C00) and np.all((got[nan] & 0x3FF) != 0)


def test_round_bf16_bit_exact():
    X = _probe_floats()
    out = torch.empty(X.shape, dtype=torch.int16, device=DEV)
    mfg.round_bf16(dev(X), out)
    got = host(out).view(np.uint16)
    ref = oracle.bf16_encode(X.astype(np.float64))
    nan = np.isnan(X)
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.all((got[nan] & 0x7F80) == 0x7F80) and np.all((got[nan] & 0x7F) != 0)


@pytest.mark.parametrize("shape", [(512, 640), (3000, 2500)])
def test_split_bit_exact_and_norms(shape):
    rng = np.random.default_rng(1)
    X = (np.where(rng.random(shape) < 0.5, -1, 1) * np.exp2(rng.uniform(-30, 15.9, shape))).astype(np.float32)
    h = torch.empty(X.shape, dtype=torch.int16, device=DEV)
    r = torch.empty(X.shape, dtype=torch.int16, device=DEV)
    norms = torch.zeros(4, dtype=torch.float64, device=DEV)
    mfg.split_f16(dev(X), h, r, norms)
    sp = oracle.split_f16(X)
    assert np.array_equal(host(h).view(np.uint16), sp.head_bits)
    assert np.array_equal(host(r).view(np.uint16), sp.resid_bits)
    x64 = X.astype(np.float64)
    res = x64 - sp.head
    n = host(norms)
    assert np.isclose(n[0], np.sum(x64 * x64), rtol=1e-12)
    assert n[1] == np.max(np.abs(x64))
    assert np.isclose(n[2], np.sum(res * res), rtol=1e-12)
    assert n[3] == np.max(np.abs(res))


@pytest.mark.parametrize("shape", [(256, 384), (300, 200), (1, 1), (129, 257)])
def test_quantize_fp8_bit_exact(shape):
    (X,) = workloads.normal(2, [shape])
    X[: min(128, shape[0]), : min(128, shape[1])] *= 300.0     # tiles with different scales
    if shape[0] > 128 and shape[1] > 128:
        X[128:, 128:] = 0.0                                     # an all-zero tile
    codes = torch.zeros(shape, dtype=torch.uint8, device=DEV)
    tr, tc = -(-shape[0] // 128), -(-shape[1] // 128)
    scales = torch.zeros((tr, tc), dtype=torch.float32, device=DEV)
    mfg.quantize_fp8(dev(X), codes, scales)
    q = oracle.fp8_quantize(X)
    assert np.array_equal(host(scales).astype(np.float64), q.scales)
    assert np.array_equal(host(codes), q.codes)


def test_e4m3_encoder_on_grid_and_midpoints():
    """All finite E4M3 values, the midpoints between them and their FP32 neighbours,
    in one tile whose scale is 1 (amax = 448)."""
    grid = np.unique(np.abs(oracle.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8))))
    mids = (grid[:-1] + grid[1:]) / 2
    pts = np.concatenate([grid, mids]).astype(np.float32)
    pts = np.concatenate([pts, np.nextafter(pts, np.float32(1e9)), np.nextafter(pts, np.float32(0))])
    pts = np.concatenate([pts, -pts, [448.0, 500.0]]).astype(np.float32)
    pts = pts[np.abs(pts) <= 448.0]
    n = pts.size
    X = np.zeros((128, 128), np.float32)
    X.flat[:n] = pts
    X[127, 127] = 448.0
    codes = torch.zeros((128, 128), dtype=torch.uint8, device=DEV)
    scales = torch.zeros((1, 1), dtype=torch.float32, device=DEV)
    mfg.quantize_fp8(dev(X), codes, scales)
    assert host(scales)[0, 0] == 1.0
    assert np.array_equal(host(codes), oracle.e4m3_encode(X.astype(np.float64)))


def test_error_norms_against_numpy():
    rng = np.random.default_rng(4)
    R = rng.standard_normal((333, 517))
    C = (R + rng.standard_normal(R.shape) * 1e-3).astype(np.float32)
    out = torch.zeros(4, dtype=torch.float64, device=DEV)
    mfg.error_norms(dev(C), dev(R), out)
    o = host(out)
    e = C.astype(np.float64) - R
    assert o[0] == np.max(np.abs(e))
    assert np.isclose(o[1], np.sqrt(np.sum(e * e)), rtol=1e-12)
    assert np.isclose(o[2], np.sqrt(np.sum(R * R)), rtol=1e-12)
    assert o[3] == np.max(np.abs(R))
    # closed form: an all-ones n x n reference against zeros has Frobenius norm n
    n = 300
    out2 = torch.zeros(4, dtype=torch.float64, device=DEV)
    mfg.error_norms(torch.zeros((n, n), device=DEV), torch.ones((n, n), dtype=torch.float64, device=DEV), out2)
    assert list(host(out2)) == [1.0, float(n), float(n), 1.0]


def test_error_norms_deterministic():
    rng = np.random.default_rng(5)
    R = rng.standard_normal((1024, 1024))
    C = R.astype(np.float32)
    outs = []
    for _ in range(3):
        o = torch.zeros(4, dtype=torch.float64, device=DEV)
        mfg.error_norms(dev(C), dev(R), o)
        outs.append(host(o))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
