"""ctypes declarations of libmfgemm's C ABI (include/mfgemm.h), same names.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfgemm.so")

# status
MFG_OK = 0
MFG_PENDING = 1
MFG_ERR_INVALID_ARG = -1
MFG_ERR_UNSUPPORTED = -2
MFG_ERR_NO_MEMORY = -3
MFG_ERR_OVER_BUDGET = -4
MFG_ERR_HIP = -5
MFG_ERR_UNKNOWN_TICKET = -6
MFG_ERR_INTERNAL = -7
# modes
MFG_F32 = 0
MFG_F16 = 1
MFG_BF16 = 2
MFG_F16_REFINE_A = 3
MFG_F16_SPLIT3 = 4
MFG_F16_SPLIT4 = 5
MFG_FP8_E4M3 = 6
MFG_BF16_SPLIT3 = 7
MFG_BF16_SPLIT6 = 8
MFG_NUM_MODES = 9
MFG_IN_PRECONVERTED = 0x100
MFG_IN_FP32 = 0x200  # grouped plans: FP32 operands, converted on every run
MFG_MODE_MASK = 0xFF
MFG_RESID_SCALE_LOG2 = 11
MFG_FP8_TILE = 128
MFG_NOALLOC_SCRATCH_BYTES = 64 << 20

MODE_BY_NAME = {
    "f32": MFG_F32, "f16": MFG_F16, "bf16": MFG_BF16, "refine_a": MFG_F16_REFINE_A,
    "split3": MFG_F16_SPLIT3, "split4": MFG_F16_SPLIT4, "fp8": MFG_FP8_E4M3, "bf16_split3": MFG_BF16_SPLIT3,
    "bf16_split6": MFG_BF16_SPLIT6,
}

i64, i32, f32, f64, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_double, ctypes.c_void_p
u64 = ctypes.c_uint64


class mfg_problem(ctypes.Structure):
    _fields_ = [("M", i64), ("N", i64), ("K", i64), ("lda", i64), ("ldb", i64), ("ldc", i64),
                ("A", vp), ("B", vp), ("C", vp)]


class mfg_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", u64), ("slots", ctypes.c_int32), ("device", ctypes.c_int32),
                ("max_group", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class mfg_request(ctypes.Structure):
    _fields_ = [("M", i64), ("N", i64), ("K", i64), ("lda", i64), ("ldb", i64), ("ldc", i64),
                ("A", vp), ("B", vp), ("C", vp), ("alpha", f32), ("beta", f32),
                ("mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class mfg_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("t_submit_ns", i64),
                ("t_admit_ns", i64), ("t_start_ns", i64), ("t_end_ns", i64), ("group_size", i64),
                ("flops", f64)]


class mfg_server_stats(ctypes.Structure):
    _fields_ = [("submitted", i64), ("completed", i64), ("failed", i64), ("launches", i64),
                ("bytes_in_use", u64), ("peak_bytes_in_use", u64), ("max_concurrent_slots", i64)]


P = ctypes.POINTER
# name -> (restype, argtypes); every symbol declared in include/mfgemm.h
SIGNATURES = {
    "mfg_fp8_scale_offset": (i64, [i64, i64]),
    "mfg_gemm": (i32, [i64, i64, i64, vp, i64, vp, i64, vp, i64, f32, f32, i32, vp]),
    "mfg_gemm_config": (i32, [i64, i64, i64, vp, i64, vp, i64, vp, i64, f32, f32, i32, i32, vp]),
    "mfg_gemm_noalloc": (i32, [i64, i64, i64, vp, i64, vp, i64, vp, i64, f32, f32, i32, vp]),
    "mfg_num_configs": (i32, [i32]),
    "mfg_config_name": (i32, [i32, i32, ctypes.c_char_p, i32]),
    "mfg_gemm_batched": (i32, [i64, i64, i64, i64, vp, i64, i64, vp, i64, i64, vp, i64, i64, f32, f32, i32, vp]),
    "mfg_grouped_plan_create": (i32, [i64, P(mfg_problem), i32, P(vp)]),
    "mfg_grouped_run": (i32, [vp, f32, f32, vp]),
    "mfg_grouped_graph_launch": (i32, [vp, f32, f32, vp]),
    "mfg_grouped_plan_info": (i32, [vp, P(f64), P(f64), P(i64)]),
    "mfg_grouped_plan_destroy": (i32, [vp]),
    "mfg_grouped_tile_classes": (i32, [i32, P(i32), i32]),
    "mfg_grouped_plan_classes": (i32, [vp, P(i32), P(i64), i32]),
    "mfg_grouped_autotune": (i32, [i64, P(mfg_problem), i32, i32, P(i32), P(f32), vp]),
    "mfg_round_f16": (i32, [i64, i64, vp, i64, vp, i64, vp]),
    "mfg_round_bf16": (i32, [i64, i64, vp, i64, vp, i64, vp]),
    "mfg_split_f16": (i32, [i64, i64, vp, i64, vp, vp, i64, vp, vp]),
    "mfg_quantize_fp8": (i32, [i64, i64, vp, i64, vp, i64, vp, vp]),
    "mfg_convert": (i32, [i64, i64, vp, i64, vp, i64, i32, vp]),
    "mfg_convert_bytes": (i64, [i64, i64, i64, i32]),
    "mfg_error_norms": (i32, [i64, i64, vp, i64, vp, i64, vp, vp]),
    "mfg_autotune": (i32, [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, i32, P(i32), P(f32), vp]),
    "mfg_tune_save": (i32, [ctypes.c_char_p]),
    "mfg_tune_load": (i32, [ctypes.c_char_p]),
    "mfg_tune_clear": (i32, []),
    "mfg_tune_lookup": (i32, [i64, i64, i64, i32]),
    "mfg_server_create": (i32, [P(mfg_server_config), P(vp)]),
    "mfg_submit": (i32, [vp, P(mfg_request), P(u64)]),
    "mfg_poll": (i32, [vp, u64, P(mfg_result)]),
    "mfg_server_drain": (i32, [vp]),
    "mfg_server_get_stats": (i32, [vp, P(mfg_server_stats)]),
    "mfg_server_destroy": (i32, [vp]),
    "mfg_status_string": (ctypes.c_char_p, [i32]),
    "mfg_last_hip_error": (i32, []),
    "mfg_version": (ctypes.c_char_p, []),
    "mfg_validate_gemm": (i32, [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32]),
    "mfg_fault_inject": (i32, [i64, i64]),
    "mfg_lu_factor": (i32, [i64, vp, i64, vp, P(i64), i32, vp]),
    "mfg_lu_solve": (i32, [i64, i64, vp, i64, vp, vp, i64, vp]),
    "mfg_solve_ir": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, i32, i32, f64, P(i32), P(f64), P(i64), vp]),
    "mfg_probe_mfma": (i32, [i32, vp, i64, i64, vp, P(f64), vp]),
}

_lib = None


class MfgError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn} failed: {status_string(status)} ({status})"
                         + (f", hip error {_lib.mfg_last_hip_error()}" if _lib and status == MFG_ERR_HIP else ""))


def lib():
    """The loaded libmfgemm (raises if the HIP library was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmfgemm not built: {LIB_PATH} is missing "
                           "(run `python -m paper_1803_04014_amd.build`)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().mfg_status_string(status).decode()


def check(fn: str, status: int) -> int:
    if status < 0:
        raise MfgError(fn, status)
    return status
