"""libmfgemm: mixed-precision GEMM on MI355X (gfx950) matrix cores.

A thin Python layer over the C ABI in include/mfgemm.h.  Every function here
only marshals arguments (torch tensors supply device memory, shapes, leading
dimensions and the current HIP stream); all arithmetic runs in the library's
HIP kernels.  The names follow the C calls without the ``mfg_`` prefix.
"""
from __future__ import annotations

import ctypes

from . import capi
from .capi import (MFG_BF16, MFG_F16, MFG_F16_REFINE_A, MFG_F16_SPLIT3, MFG_F16_SPLIT4, MFG_F32,
                   MFG_FP8_E4M3, MFG_IN_PRECONVERTED, MODE_BY_NAME, MfgError, check, lib)

__all__ = [
    "MFG_F32", "MFG_F16", "MFG_BF16", "MFG_F16_REFINE_A", "MFG_F16_SPLIT3", "MFG_F16_SPLIT4",
    "MFG_FP8_E4M3", "MFG_IN_PRECONVERTED", "MODE_BY_NAME", "MfgError", "lib", "mode_of",
    "gemm", "gemm_batched", "GroupedPlan", "round_f16", "round_bf16", "split_f16", "quantize_fp8",
    "convert", "convert_bytes", "error_norms", "autotune", "num_configs", "config_name", "Server",
]


def mode_of(mode) -> int:
    return MODE_BY_NAME[mode] if isinstance(mode, str) else int(mode)


def _stream(stream=None) -> int:
    import torch

    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libmfgemm operates on device (HIP) tensors")
    return ctypes.c_void_p(t.data_ptr())


def _ld(t) -> int:
    if t.dim() == 2 and t.numel() == 0:
        return max(1, t.shape[1])
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("expected a 2-D row-major tensor with unit column stride")
    return max(1, t.stride(0))


def gemm(A, B, C, alpha: float = 1.0, beta: float = 0.0, mode="f16", preconverted: bool = False,
         M: int | None = None, K: int | None = None, config: int = -1, stream=None) -> None:
    """mfg_gemm / mfg_gemm_config: C = alpha*A*B + beta*C in `mode`, in place.

    With ``preconverted`` the operands are in the mode's storage form (as written
    by :func:`convert`); then ``M`` and ``K`` give the logical sizes when the
    tensors carry extra planes (split residuals, FP8 scales).
    """
    m = mode_of(mode) | (MFG_IN_PRECONVERTED if preconverted else 0)
    Mv = C.shape[0] if M is None else M
    N = C.shape[1]
    Kv = (A.shape[1] if K is None else K)
    s = _stream(stream)
    st = lib().mfg_gemm_config(Mv, N, Kv, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C),
                               float(alpha), float(beta), m, int(config), ctypes.c_void_p(s))
    check("mfg_gemm", st)


def gemm_batched(A, B, C, alpha: float = 1.0, beta: float = 0.0, mode="f16", preconverted: bool = False,
                 M: int | None = None, K: int | None = None, stream=None) -> None:
    """mfg_gemm_batched over 3-D tensors (batch, rows, cols), row-major entries.

    With ``preconverted`` each entry holds the mode's storage form (head plane,
    then residual plane); ``M`` and ``K`` then give the logical sizes."""
    cnt = A.shape[0]
    Mv = C.shape[1] if M is None else M
    Kv = A.shape[2] if K is None else K
    N = C.shape[2]
    for t in (A, B, C):
        if t.dim() != 3 or t.stride(2) != 1:
            raise ValueError("expected 3-D tensors with unit innermost stride")
    m = mode_of(mode) | (MFG_IN_PRECONVERTED if preconverted else 0)
    st = lib().mfg_gemm_batched(cnt, Mv, N, Kv, _ptr(A), max(1, A.stride(1)), A.stride(0), _ptr(B),
                                max(1, B.stride(1)), B.stride(0), _ptr(C), max(1, C.stride(1)), C.stride(0),
                                float(alpha), float(beta), m, ctypes.c_void_p(_stream(stream)))
    check("mfg_gemm_batched", st)


def lu_factor(A, mode="f32", stream=None):
    """mfg_lu_factor on a square FP32 device tensor, in place: returns (ipiv int32 device tensor, info)."""
    import torch

    n = A.shape[0]
    ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    info = ctypes.c_int64()
    check("mfg_lu_factor", lib().mfg_lu_factor(n, _ptr(A), _ld(A), _ptr(ipiv), ctypes.byref(info), mode_of(mode),
                                               ctypes.c_void_p(_stream(stream))))
    return ipiv[:n], info.value


def lu_solve(LU, ipiv, B, stream=None):
    """mfg_lu_solve: B (n x nrhs FP32 device tensor) = (L U)^-1 P B in place."""
    check("mfg_lu_solve", lib().mfg_lu_solve(LU.shape[0], B.shape[1], _ptr(LU), _ld(LU), _ptr(ipiv), _ptr(B), _ld(B),
                                             ctypes.c_void_p(_stream(stream))))


def solve_ir(A, B, X, mode="f32", max_iter=10, tol=2.0 ** -50, stream=None):
    """mfg_solve_ir on FP64 device tensors A (n x n), B and X (n x nrhs): returns
    {"iters", "berr", "info"}."""
    it, be, info = ctypes.c_int(), ctypes.c_double(), ctypes.c_int64()
    check("mfg_solve_ir", lib().mfg_solve_ir(A.shape[0], B.shape[1], _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(X), _ld(X),
                                             mode_of(mode), int(max_iter), float(tol), ctypes.byref(it),
                                             ctypes.byref(be), ctypes.byref(info), ctypes.c_void_p(_stream(stream))))
    return {"iters": it.value, "berr": be.value, "info": info.value}


def _problems(problems):
    """(A, B, C) device tensors -> a ctypes mfg_problem array."""
    arr = (capi.mfg_problem * len(problems))()
    for i, (A, B, C) in enumerate(problems):
        M, K = A.shape
        N = B.shape[1]
        arr[i] = capi.mfg_problem(M, N, K, _ld(A), _ld(B), _ld(C), A.data_ptr(), B.data_ptr(), C.data_ptr())
    return arr


def grouped_tile_classes(mode="f16"):
    """mfg_grouped_tile_classes: the grouped kernel's tile sides for `mode`, the default first."""
    t = (ctypes.c_int * 4)()
    n = check("mfg_grouped_tile_classes", lib().mfg_grouped_tile_classes(mode_of(mode), t, 4))
    return [t[i] for i in range(n)]


def grouped_autotune(problems, mode="f16", fp32_in=False, reps=5, stream=None):
    """mfg_grouped_autotune over (A, B, C) problems of one size bucket: (best tile side, ms per run)."""
    arr = _problems(problems)
    best, ms = ctypes.c_int(), ctypes.c_float()
    m = mode_of(mode) | (capi.MFG_IN_FP32 if fp32_in else 0)
    check("mfg_grouped_autotune", lib().mfg_grouped_autotune(len(problems), arr, m, int(reps), ctypes.byref(best),
                                                             ctypes.byref(ms), ctypes.c_void_p(_stream(stream))))
    return best.value, ms.value


class GroupedPlan:
    """mfg_grouped_plan_*: many GEMMs of different shapes in one persistent launch."""

    def __init__(self, problems, mode="f16", fp32_in=False):
        """`problems`: list of (A, B, C) 2-D device tensors (A: M x K, B: K x N, C: M x N); A and B
        in the mode's preconverted form, or FP32 with `fp32_in` (MFG_IN_FP32)."""
        arr = _problems(problems)
        self._keep = list(problems)
        h = ctypes.c_void_p()
        m = mode_of(mode) | (capi.MFG_IN_FP32 if fp32_in else 0)
        check("mfg_grouped_plan_create", lib().mfg_grouped_plan_create(len(problems), arr, m, ctypes.byref(h)))
        self.handle = h

    def run(self, alpha=1.0, beta=0.0, stream=None):
        check("mfg_grouped_run", lib().mfg_grouped_run(self.handle, alpha, beta, ctypes.c_void_p(_stream(stream))))

    def graph_launch(self, alpha=1.0, beta=0.0, stream=None):
        check("mfg_grouped_graph_launch",
              lib().mfg_grouped_graph_launch(self.handle, alpha, beta, ctypes.c_void_p(_stream(stream))))

    def info(self):
        f, b, w = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        check("mfg_grouped_plan_info", lib().mfg_grouped_plan_info(self.handle, ctypes.byref(f), ctypes.byref(b),
                                                                   ctypes.byref(w)))
        return {"flops": f.value, "bytes": b.value, "work_items": w.value}

    def classes(self):
        """{tile side: work items} of the classes this plan launches."""
        t, n = (ctypes.c_int * 2)(), (ctypes.c_int64 * 2)()
        k = check("mfg_grouped_plan_classes", lib().mfg_grouped_plan_classes(self.handle, t, n, 2))
        return {t[i]: n[i] for i in range(k)}

    def close(self):
        if getattr(self, "handle", None):
            lib().mfg_grouped_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def round_f16(X, out, stream=None):
    check("mfg_round_f16", lib().mfg_round_f16(X.shape[0], X.shape[1], _ptr(X), _ld(X), _ptr(out), _ld(out),
                                               ctypes.c_void_p(_stream(stream))))


def round_bf16(X, out, stream=None):
    check("mfg_round_bf16", lib().mfg_round_bf16(X.shape[0], X.shape[1], _ptr(X), _ld(X), _ptr(out), _ld(out),
                                                 ctypes.c_void_p(_stream(stream))))


def split_f16(X, head, resid, norms=None, stream=None):
    check("mfg_split_f16", lib().mfg_split_f16(X.shape[0], X.shape[1], _ptr(X), _ld(X), _ptr(head), _ptr(resid),
                                               _ld(head), _ptr(norms), ctypes.c_void_p(_stream(stream))))


def quantize_fp8(X, codes, scales, stream=None):
    check("mfg_quantize_fp8", lib().mfg_quantize_fp8(X.shape[0], X.shape[1], _ptr(X), _ld(X), _ptr(codes),
                                                     _ld(codes), _ptr(scales), ctypes.c_void_p(_stream(stream))))


def convert_bytes(rows: int, cols: int, ldo: int, mode) -> int:
    return int(lib().mfg_convert_bytes(rows, cols, ldo, mode_of(mode)))


def convert(X, out, ldo: int, mode, stream=None):
    """mfg_convert: write X in `mode`'s preconverted storage form into the byte buffer `out`."""
    check("mfg_convert", lib().mfg_convert(X.shape[0], X.shape[1], _ptr(X), _ld(X), _ptr(out), ldo, mode_of(mode),
                                           ctypes.c_void_p(_stream(stream))))


def error_norms(C, Cref, out4, stream=None):
    check("mfg_error_norms", lib().mfg_error_norms(C.shape[0], C.shape[1], _ptr(C), _ld(C), _ptr(Cref), _ld(Cref),
                                                   _ptr(out4), ctypes.c_void_p(_stream(stream))))


def autotune(A, B, C, mode, reps=3, preconverted=False, M=None, K=None, stream=None):
    m = mode_of(mode) | (MFG_IN_PRECONVERTED if preconverted else 0)
    Mv = C.shape[0] if M is None else M
    Kv = A.shape[1] if K is None else K
    best, ms = ctypes.c_int(), ctypes.c_float()
    check("mfg_autotune", lib().mfg_autotune(Mv, C.shape[1], Kv, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C),
                                             m, reps, ctypes.byref(best), ctypes.byref(ms),
                                             ctypes.c_void_p(_stream(stream))))
    return best.value, ms.value


def num_configs(mode) -> int:
    return int(lib().mfg_num_configs(mode_of(mode)))


def config_name(mode, cfg: int) -> str:
    buf = ctypes.create_string_buffer(64)
    check("mfg_config_name", lib().mfg_config_name(mode_of(mode), cfg, buf, 64))
    return buf.value.decode()


class Server:
    """mfg_server_*: continuous-batching request loop with HBM admission."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 4, device: int = 0, max_group: int = 16):
        cfg = capi.mfg_server_config(int(hbm_budget_bytes), slots, device, max_group, 0)
        h = ctypes.c_void_p()
        check("mfg_server_create", lib().mfg_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def submit(self, A, B, C, mode, alpha=1.0, beta=0.0, M=None, N=None, K=None, A_ptr=None, B_ptr=None,
               C_ptr=None, lda=None, ldb=None, ldc=None) -> int:
        """Submit C = alpha*A*B + beta*C; returns the ticket.  Views may be given as
        tensors or as raw (pointer, ld) pairs for sub-blocks of larger pools."""
        Mv = M if M is not None else C.shape[0]
        Nv = N if N is not None else C.shape[1]
        Kv = K if K is not None else A.shape[1]
        req = capi.mfg_request(Mv, Nv, Kv, lda or _ld(A), ldb or _ld(B), ldc or _ld(C),
                               A_ptr or A.data_ptr(), B_ptr or B.data_ptr(), C_ptr or C.data_ptr(),
                               float(alpha), float(beta), mode_of(mode), 0)
        t = ctypes.c_uint64()
        check("mfg_submit", lib().mfg_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """Returns (status, result-dict); status MFG_PENDING (1) while running."""
        r = capi.mfg_result()
        st = lib().mfg_poll(self.handle, ticket, ctypes.byref(r))
        return st, {f: getattr(r, f) for f, _ in capi.mfg_result._fields_}

    def drain(self):
        check("mfg_server_drain", lib().mfg_server_drain(self.handle))

    def stats(self):
        s = capi.mfg_server_stats()
        check("mfg_server_get_stats", lib().mfg_server_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in capi.mfg_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().mfg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
