"""The matrix-core ceiling probe (mfg_probe_mfma) on known operands.

With every operand equal to 1, each MFMA adds its depth K to every output it
accumulates, so after `iters` rounds of the probe's 8 independent chains each
lane's sum of its accumulators is exactly 8 * (outputs per lane) * iters * K:
16 outputs and K = 16 for the 32x32x16 FP16 shape, 4 and 32 for 16x16x32 FP16,
16 and 64 for the 32x32x64 E4M3 shape (unit scales).  The reported flops are
the instruction's 2 * 32 * 32 * K (or 2 * 16 * 16 * 32) per MFMA.
"""
import ctypes

import pytest
import torch

import paper_1803_04014_amd as mfg
from gpu_util import DEV, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,outs,k,mnk", [(0, 16, 16, 32 * 32 * 16), (1, 4, 32, 16 * 16 * 32),
                                              (2, 16, 64, 32 * 32 * 64)])
def test_probe_sums_on_ones(shape, outs, k, mnk):
    need_gpu()
    if shape == 2:
        ops = torch.ones(16384, dtype=torch.float32, device=DEV).to(torch.float8_e4m3fn).view(torch.uint8)
    else:
        ops = torch.ones(8192, dtype=torch.float16, device=DEV)
    wg, iters = 3, 5
    out = torch.full((wg * 256,), float("nan"), dtype=torch.float32, device=DEV)
    fl = ctypes.c_double()
    st = mfg.lib().mfg_probe_mfma(shape, ctypes.c_void_p(ops.data_ptr()), wg, iters, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.byref(fl), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    want = 8 * outs * iters * k
    assert torch.all(out == want), (shape, out[:4].tolist(), want)
    assert fl.value == 2.0 * mnk * 8 * iters * wg * 4
