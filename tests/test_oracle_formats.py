"""Pins of the oracle's number formats against independent routines and the paper.

* FP16: numpy's IEEE binary16 conversion (an independent library routine) over
  every half value, its neighbours and every rounding midpoint, plus random
  FP32 bit patterns; and the facts the paper states in Sec. V.
* BF16: torch's CPU float->bfloat16 cast (round to nearest even).
* FP8 E4M3: torch's CPU float8_e4m3fn cast on in-range values, and the
  format's defining constants (max 448, NaN code, subnormal spacing).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _np_f16_bits(x32):
    return np.asarray(x32, np.float32).astype(np.float16).view(np.uint16)


def _same_bits_or_both_nan(a_bits, b_bits, isnan):
    ok = (a_bits == b_bits) | isnan
    return bool(np.all(ok))


def test_f16_decode_all_codes():
    codes = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ours = oracle.f16_decode(codes)
    ref = codes.view(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])


def _f16_probe_points():
    """Every finite half value, its FP32 neighbours, every midpoint between adjacent
    halves and the FP32 neighbours of those midpoints (both signs)."""
    codes = np.arange(0, 0x7C00, dtype=np.uint32).astype(np.uint16)  # +0 .. max finite
    vals = codes.view(np.float16).astype(np.float32)
    nxt = np.append(vals[1:], np.float32(65536.0))  # the next grid point above max is 2^16
    mids = ((vals.astype(np.float64) + nxt.astype(np.float64)) / 2).astype(np.float32)
    pts = [vals, mids]
    for base in (vals, mids):
        pts.append(np.nextafter(base, np.float32(np.inf)))
        pts.append(np.nextafter(base, np.float32(-np.inf)))
    p = np.concatenate(pts).astype(np.float32)
    p = p[np.isfinite(p)]
    return np.concatenate([p, -p])


def test_f16_encode_matches_numpy_on_all_midpoints():
    x = _f16_probe_points()
    ours = oracle.f16_encode(x.astype(np.float64))
    ref = _np_f16_bits(x)
    assert _same_bits_or_both_nan(ours, ref, np.zeros_like(ours, bool))


def test_f16_encode_matches_numpy_on_random_bit_patterns():
    rng = np.random.default_rng(123)
    bits = rng.integers(0, 2 ** 32, size=2_000_000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    ours = oracle.f16_encode(x.astype(np.float64))
    ref = _np_f16_bits(x)
    isnan = np.isnan(x)
    assert _same_bits_or_both_nan(ours, ref, isnan)
    # NaN stays NaN
    assert np.all(np.isnan(oracle.f16_decode(ours[isnan])))


def test_f16_paper_facts():
    """Sec. V: max 65504, larger values become infinity, 1024 values per binade,
    spacing 2^-10 at 1 and 32 in [2^15, 2^16), tiny values become zero."""
    with open(os.path.join(GOLDEN, "paper_fp16_facts.json")) as f:
        facts = json.load(f)
    enc, dec = oracle.f16_encode, oracle.f16_decode
    assert dec(np.array([0x7BFF], np.uint16))[0] == facts["max_finite"]
    # 65504 is representable; the overflow threshold is the midpoint to 2^16
    assert enc(np.array([65504.0]))[0] == 0x7BFF
    assert enc(np.array([65519.996]))[0] == 0x7BFF
    assert enc(np.array([65520.0]))[0] == 0x7C00
    assert enc(np.array([1e6]))[0] == 0x7C00
    assert enc(np.array([-1e6]))[0] == 0xFC00
    # values per power-of-two interval
    for lo in facts["binades_with_1024_values"]:
        c0 = enc(np.array([float(lo)]))[0]
        c1 = enc(np.array([float(2 * lo)]))[0]
        assert int(c1) - int(c0) == facts["values_per_binade"]
    # spacing at 1 (machine epsilon 2^-10) and in [2^15, 2^16)
    assert dec(np.array([0x3C01], np.uint16))[0] - 1.0 == facts["spacing_at_1"]
    a = dec(np.array([enc(np.array([32768.0]))[0]], np.uint16))[0]
    b = dec(np.array([enc(np.array([32768.0]))[0] + 1], np.uint16))[0]
    assert b - a == facts["spacing_2p15_2p16"]
    # all fractional precision is lost above 1024
    assert dec(enc(np.array([1024.4])))[0] == 1024.0
    # too small to represent -> zero (below half the smallest subnormal 2^-24)
    assert enc(np.array([2.0 ** -26]))[0] == 0
    assert enc(np.array([2.0 ** -25]))[0] == 0          # tie, rounds to even (zero)
    assert enc(np.array([2.0 ** -25 * 1.0001]))[0] == 1  # just above the tie
    assert dec(np.array([1], np.uint16))[0] == 2.0 ** -24


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(7)
    bits = rng.integers(0, 2 ** 32, size=1_000_000, dtype=np.uint64).astype(np.uint32)
    x = np.concatenate([bits.view(np.float32),
                        rng.standard_normal(200_000).astype(np.float32),
                        np.array([0.0, -0.0, 3.3895314e38, -3.3895314e38, 1e-40, np.inf, -np.inf],
                                 np.float32)])
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    ours = oracle.bf16_encode(x.astype(np.float64))
    isnan = np.isnan(x)
    assert _same_bits_or_both_nan(ours, ref, isnan)
    dec = oracle.bf16_decode(ours[~isnan])
    tdec = torch.from_numpy(ref[~isnan].view(np.int16).copy()).view(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(dec, tdec)


def test_e4m3_decode_table():
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.e4m3_decode(codes)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])
    assert set(np.flatnonzero(nan).tolist()) == {0x7F, 0xFF}
    assert np.nanmax(ours) == 448.0
    assert ours[1] == 2.0 ** -9      # smallest subnormal
    assert ours[8] == 2.0 ** -6      # smallest normal


def test_e4m3_encode_matches_torch_in_range():
    rng = np.random.default_rng(11)
    x = np.concatenate([
        rng.uniform(-448, 448, 300_000),
        rng.standard_normal(300_000) * 2.0 ** rng.integers(-12, 8, 300_000),
        oracle.e4m3_decode(np.arange(256, dtype=np.uint8)),  # grid points
    ])
    x = x[np.isfinite(x) & (np.abs(x) <= 448.0)].astype(np.float32)  # torch does not saturate
    # midpoints between adjacent positive grid values (ties go to even)
    grid = np.sort(np.unique(oracle.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8))))
    mids = ((grid[:-1] + grid[1:]) / 2).astype(np.float32)
    x = np.concatenate([x, mids, -mids])
    ours = oracle.e4m3_encode(x.astype(np.float64))
    ref = torch.from_numpy(x.copy()).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_saturates():
    v = oracle.e4m3_encode(np.array([448.0, 463.9, 464.0, 500.0, 1e9, -1e9, np.inf, -np.inf]))
    assert list(v) == [0x7E, 0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0x7E, 0xFE]
