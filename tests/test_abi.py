"""The C-ABI boundary on the CPU: the built libmfgemm exports every function
include/mfgemm.h declares, the Python binding declares the same names, the
numeric constants and struct layouts agree with the header, and the host-only
entry points (validation, sizes, names, tuned table) behave as documented.
No call here touches a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1803_04014_amd as mfg
from paper_1803_04014_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfgemm.h")


def header_text():
    with open(HEADER) as f:
        return f.read()


def declared_functions():
    src = re.sub(r"/\*.*?\*/", "", header_text(), flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(mfg_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_documented_calls():
    names = declared_functions()
    for must in ("mfg_gemm", "mfg_gemm_batched", "mfg_submit", "mfg_poll", "mfg_error_norms", "mfg_split_f16",
                 "mfg_quantize_fp8", "mfg_grouped_graph_launch", "mfg_autotune", "mfg_server_create"):
        assert must in names
    assert len(names) >= 30


def test_library_exports_every_declared_symbol():
    lib = mfg.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\sT\s+(mfg_[a-z_0-9]+)$", out.stdout, flags=re.M))
    assert set(declared_functions()) <= exported
    # nothing else of the C ABI leaks out under the mfg_ prefix
    assert exported - set(declared_functions()) == set()


def test_binding_declares_exactly_the_header():
    assert set(capi.SIGNATURES) == set(declared_functions())


def test_constants_match_header():
    src = header_text()
    values = {k: int(v, 0) for k, v in re.findall(r"#define\s+(MFG_[A-Z0-9_]+)\s+(0x[0-9A-Fa-f]+|-?\d+)", src)}
    values.update({k: int(v) for k, v in re.findall(r"\b(MFG_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)})
    assert len(values) >= 20
    for k, v in values.items():
        assert getattr(capi, k) == v, k


def test_struct_layouts():
    assert ctypes.sizeof(capi.mfg_problem) == 6 * 8 + 3 * 8
    assert ctypes.sizeof(capi.mfg_server_config) == 8 + 4 * 4
    assert ctypes.sizeof(capi.mfg_request) == 6 * 8 + 3 * 8 + 4 * 4
    assert ctypes.sizeof(capi.mfg_result) == 4 + 4 + 5 * 8 + 8
    assert ctypes.sizeof(capi.mfg_server_stats) == 7 * 8


def test_version_and_status_strings():
    assert mfg.lib().mfg_version().decode().startswith("libmfgemm")
    for st in range(-7, 2):
        assert mfg.lib().mfg_status_string(st)
    assert b"unknown" in mfg.lib().mfg_status_string(-99).lower()


P = 0x7F0000000000  # a non-null address: validation never dereferences


@pytest.mark.parametrize("args,expect", [
    ((8, 8, 8, P, 8, P, 8, P, 8, 1), 0),
    ((0, 8, 8, None, 8, P, 8, None, 8, 1), 0),              # M = 0: A and C have no extent
    ((8, 8, 0, None, 1, None, 8, P, 8, 1), 0),              # K = 0: A, B unused
    ((-1, 8, 8, P, 8, P, 8, P, 8, 1), -1),
    ((8, 8, 8, P, 7, P, 8, P, 8, 1), -1),                   # lda < K
    ((8, 8, 8, P, 8, P, 7, P, 8, 1), -1),                   # ldb < N
    ((8, 8, 8, P, 8, P, 8, P, 7, 1), -1),                   # ldc < N
    ((8, 8, 8, None, 8, P, 8, P, 8, 1), -1),
    ((8, 8, 8, P, 8, P, 8, None, 8, 1), -1),
    ((8, 8, 8, P, 8, P, 8, P, 8, 8), 0),                    # MFG_BF16_SPLIT6
    ((8, 8, 8, P, 8, P, 8, P, 8, 9), -1),                   # no such mode
    ((8, 8, 8, P, 8, P, 8, P, 8, 0x201), -1),               # unknown flag
    ((8, 8, 8, P, 8, P, 8, P, 8, 0x101), 0),
])
def test_validation_rules(args, expect):
    assert mfg.lib().mfg_validate_gemm(*args) == expect


def test_convert_bytes_and_fp8_scale_offset():
    L = mfg.lib()
    assert L.mfg_convert_bytes(10, 7, 8, capi.MFG_F16) == 10 * 8 * 2
    assert L.mfg_convert_bytes(10, 7, 8, capi.MFG_F16_SPLIT3) == 2 * 10 * 8 * 2
    assert L.mfg_convert_bytes(10, 7, 8, capi.MFG_BF16_SPLIT3) == 2 * 10 * 8 * 2
    assert L.mfg_convert_bytes(10, 7, 8, capi.MFG_NUM_MODES) == -1
    assert L.mfg_convert_bytes(10, 7, 8, capi.MFG_BF16_SPLIT6) == -1  # no preconverted form
    assert L.mfg_convert_bytes(10, 7, 8, capi.MFG_F32) == 10 * 8 * 4
    off = L.mfg_fp8_scale_offset(300, 272)
    assert off >= 300 * 272 and off % 16 == 0
    assert L.mfg_convert_bytes(300, 260, 272, capi.MFG_FP8_E4M3) == off + 4 * 3 * 3


def test_config_menus_and_names():
    for mode in mfg.capi.MODE_BY_NAME:
        n = mfg.num_configs(mode)
        assert n >= 1
        names = [mfg.config_name(mode, i) for i in range(n)]
        assert len(set(names)) == n and all(names)
        assert mfg.lib().mfg_config_name(capi.MODE_BY_NAME[mode], n, ctypes.create_string_buffer(64), 64) != 0


def test_grouped_tile_classes_and_tuned_entries(tmp_path):
    L = mfg.lib()
    assert mfg.grouped_tile_classes("f16") == [128, 64] and mfg.grouped_tile_classes("bf16") == [128, 64]
    for m in ("refine_a", "split3", "bf16_split3"):
        assert mfg.grouped_tile_classes(m) == [64, 128]
    assert mfg.grouped_tile_classes("split4") == [64]
    t = (ctypes.c_int * 2)()
    for m in ("f32", "fp8", "bf16_split6"):
        assert L.mfg_grouped_tile_classes(capi.MODE_BY_NAME[m], t, 2) == capi.MFG_ERR_UNSUPPORTED
    assert L.mfg_grouped_tile_classes(capi.MFG_F16, None, 2) == capi.MFG_ERR_INVALID_ARG
    assert L.mfg_grouped_tile_classes(capi.MFG_F16, t, 0) == capi.MFG_ERR_INVALID_ARG
    # grouped entries live at mode 32 + mode; modes beyond either range are rejected
    L.mfg_tune_clear()
    good = tmp_path / "g.txt"
    good.write_text(f"{32 + capi.MFG_F16} 6 6 7 64\n{32 + capi.MFG_F16_SPLIT3} 8 8 8 128\n")
    assert L.mfg_tune_load(str(good).encode()) == 0
    out = tmp_path / "o.txt"
    assert L.mfg_tune_save(str(out).encode()) == 0
    rows = [ln.split() for ln in out.read_text().splitlines() if ln.strip() and not ln.startswith("#")]
    assert ["33", "6", "6", "7", "64"] in rows and ["36", "8", "8", "8", "128"] in rows
    for bad_mode in (31, 32 + capi.MFG_NUM_MODES):
        bad = tmp_path / f"b{bad_mode}.txt"
        bad.write_text(f"{bad_mode} 1 1 1 64\n")
        assert L.mfg_tune_load(str(bad).encode()) == capi.MFG_ERR_INVALID_ARG
    L.mfg_tune_clear()
    # the tuner's argument checks come before any device work
    best, ms = ctypes.c_int(), ctypes.c_float()
    arr = (capi.mfg_problem * 1)()
    assert L.mfg_grouped_autotune(0, arr, capi.MFG_F16, 3, ctypes.byref(best), ctypes.byref(ms), None) == \
        capi.MFG_ERR_INVALID_ARG
    assert L.mfg_grouped_autotune(1, arr, capi.MFG_F16, 0, ctypes.byref(best), ctypes.byref(ms), None) == \
        capi.MFG_ERR_INVALID_ARG
    assert L.mfg_grouped_autotune(1, arr, capi.MFG_F32, 3, ctypes.byref(best), ctypes.byref(ms), None) == \
        capi.MFG_ERR_UNSUPPORTED


def test_shipped_tuned_table_loads_and_names_valid_configs():
    """The table shipped with the package (written on an MI355X by
    bench.py --write-tune-table) loads, and every entry it holds names a
    configuration (GEMM) or tile class (grouped) the mode has."""
    import os
    path = os.path.join(os.path.dirname(mfg.__file__), "tuned", "mi355x_gfx950.txt")
    L = mfg.lib()
    L.mfg_tune_clear()
    assert L.mfg_tune_load(path.encode()) == 0
    L.mfg_tune_clear()
    n_gemm = n_grouped = 0
    for ln in open(path):
        if not ln.strip() or ln.startswith("#"):
            continue
        mode, mb, nb, kb, cfg = (int(x) for x in ln.split())
        if mode >= 32:
            assert cfg in mfg.grouped_tile_classes(mode - 32)
            n_grouped += 1
        else:
            assert 0 <= cfg < mfg.num_configs(mode)
            n_gemm += 1
    assert n_gemm >= 4 and n_grouped >= 2


def test_tuned_table_round_trip(tmp_path):
    L = mfg.lib()
    L.mfg_tune_clear()
    base = L.mfg_tune_lookup(4096, 4096, 4096, capi.MFG_F16)
    assert 0 <= base < mfg.num_configs("f16")
    path = tmp_path / "tuned.txt"
    path.write_text(f"{capi.MFG_F16} 12 12 12 3\n")
    assert L.mfg_tune_load(str(path).encode()) == 0
    got = [L.mfg_tune_lookup(n, n, n, capi.MFG_F16) for n in (4096, 8192)]
    assert 3 in got
    out = tmp_path / "saved.txt"
    assert L.mfg_tune_save(str(out).encode()) == 0
    rows = [ln.split() for ln in out.read_text().splitlines() if ln.strip() and not ln.startswith("#")]
    assert rows == [f"{capi.MFG_F16} 12 12 12 3".split()]
    L.mfg_tune_clear()
    assert L.mfg_tune_lookup(4096, 4096, 4096, capi.MFG_F16) == base


def test_grouped_plan_rejects_bad_modes_before_any_device_call():
    """Mode and flag checks of mfg_grouped_plan_create come before any HIP call:
    unknown flags and MFG_IN_FP32 together with MFG_IN_PRECONVERTED are
    invalid, FP32 and FP8 plans unsupported, and `out` is cleared."""
    L = mfg.lib()
    probs = (capi.mfg_problem * 1)()
    probs[0] = capi.mfg_problem(8, 8, 8, 8, 8, 8, P, P, P)
    h = ctypes.c_void_p(1234)
    cases = [
        (capi.MFG_F16 | capi.MFG_IN_FP32 | capi.MFG_IN_PRECONVERTED, capi.MFG_ERR_INVALID_ARG),
        (capi.MFG_F16 | 0x400, capi.MFG_ERR_INVALID_ARG),
        (99, capi.MFG_ERR_INVALID_ARG),
        (capi.MFG_F32, capi.MFG_ERR_UNSUPPORTED),
        (capi.MFG_FP8_E4M3 | capi.MFG_IN_FP32, capi.MFG_ERR_UNSUPPORTED),
    ]
    for mode, expect in cases:
        h.value = 1234
        assert L.mfg_grouped_plan_create(1, probs, mode, ctypes.byref(h)) == expect, hex(mode)
        assert not h.value
    assert L.mfg_grouped_plan_create(-1, probs, capi.MFG_F16, ctypes.byref(h)) == capi.MFG_ERR_INVALID_ARG
    # MFG_IN_FP32 is a grouped-plan flag only: the single GEMM's validation rejects it
    assert L.mfg_validate_gemm(8, 8, 8, P, 8, P, 8, P, 8, capi.MFG_F16 | capi.MFG_IN_FP32) == capi.MFG_ERR_INVALID_ARG


def test_batched_validates_mode_flags_before_any_device_call():
    """mfg_gemm_batched checks the whole mode: only MFG_IN_PRECONVERTED may
    accompany it (implied for F16 / BF16 / F32, the preconverted planes for
    the refined modes); FP8 is unsupported.  count = 0 returns before any
    device call once the arguments are valid."""
    L = mfg.lib()

    def call(count, mode):
        return L.mfg_gemm_batched(count, 8, 8, 8, P, 8, 64, P, 8, 64, P, 8, 64, 1.0, 0.0, mode, None)

    assert call(1, capi.MFG_F16 | capi.MFG_IN_FP32) == capi.MFG_ERR_INVALID_ARG
    assert call(1, capi.MFG_F16_SPLIT3 | capi.MFG_IN_FP32) == capi.MFG_ERR_INVALID_ARG
    assert call(1, capi.MFG_F16_SPLIT3 | 0x400) == capi.MFG_ERR_INVALID_ARG
    assert call(1, 99) == capi.MFG_ERR_INVALID_ARG
    assert call(1, capi.MFG_FP8_E4M3) == capi.MFG_ERR_UNSUPPORTED
    assert call(1, capi.MFG_FP8_E4M3 | capi.MFG_IN_PRECONVERTED) == capi.MFG_ERR_UNSUPPORTED
    for m in ("f16", "bf16", "f32", "refine_a", "split3", "split4", "bf16_split3"):
        assert call(0, capi.MODE_BY_NAME[m]) == capi.MFG_OK
        assert call(0, capi.MODE_BY_NAME[m] | capi.MFG_IN_PRECONVERTED) == capi.MFG_OK


def test_fault_inject_arguments():
    L = mfg.lib()
    assert L.mfg_fault_inject(-1, 0) == capi.MFG_ERR_INVALID_ARG
    assert L.mfg_fault_inject(0, -3) == capi.MFG_ERR_INVALID_ARG
    assert L.mfg_fault_inject(0, 0) == capi.MFG_OK


def test_probe_mfma_arguments():
    L = mfg.lib()
    f = ctypes.c_double()
    assert L.mfg_probe_mfma(3, P, 1, 1, P, ctypes.byref(f), None) == capi.MFG_ERR_INVALID_ARG
    assert L.mfg_probe_mfma(-1, P, 1, 1, P, ctypes.byref(f), None) == capi.MFG_ERR_INVALID_ARG
    assert L.mfg_probe_mfma(0, None, 1, 1, P, ctypes.byref(f), None) == capi.MFG_ERR_INVALID_ARG
    assert L.mfg_probe_mfma(0, P, 0, 1, P, ctypes.byref(f), None) == capi.MFG_ERR_INVALID_ARG
    assert L.mfg_probe_mfma(1, P, 1, 0, P, ctypes.byref(f), None) == capi.MFG_ERR_INVALID_ARG
