#!/usr/bin/env python3
"""Benchmark of libmfgemm on one MI355X.

Headline step: one FP16-in / FP32-accumulate GEMM  C = A B + C  at
M = N = K = 8192 (alpha = beta = 1, row-major), the size at which the paper
reports its best matrix-unit GEMM (Sec. VII.A).  A and B are FP32 uniform in
[-1, 1] rounded to FP16 before timing (the paper leaves the rounding out of
its timings, Sec. VI); C0 is uniform in [-1, 1].  Inputs are resident in HBM
when the timed region starts.

Prints ONE JSON line.  Besides the headline it carries:
  roofline      the GEMM kernel's average launch time (HIP events on the
                stream it runs on) against the dense FP16 MFMA peak;
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of rows of the
                same GEMM (the rows it computes also give the FP64 reference
                for the error figures);
  errors        max and Frobenius relative error vs FP64 on those rows, for
                FP16, the split-refined mode and FP32 (reduced on the GPU);
  extras        BF16 / FP32 / refined / FP8 rates at 8192, an N sweep, the
                batched and grouped workloads (GEMM/s, % of HBM roofline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TFLOP/s and % MFMA peak at max-rel-err vs FP64; batched GEMM/s; p50/p99 latency"
PEAK_TFLOPS = {"f16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "f32": 157.3}
HBM_GBS = 8000.0
PAPER_V100_TFLOPS = 83.0   # best mixed-precision GEMM on V100, N=8192 (context)
KERNEL_SOURCES = ["paper_1803_04014_amd/csrc/tile16.h", "paper_1803_04014_amd/csrc/fast16.h",
                  "paper_1803_04014_amd/csrc/pipe16.h", "paper_1803_04014_amd/csrc/gemm16.hip",
                  "paper_1803_04014_amd/csrc/device.h"]
PMC_FILE = os.path.join(ROOT, "profiles", "gemm_f16_n8192_pmc.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, reps, warm=2):
    """Average milliseconds of fn() over reps launches, HIP events on the current stream."""
    import torch

    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def grouped_legs(timed, dev) -> dict:
    """Grouped plans over 4096 problems, M, N, K log-uniform in [16, 512] (seed 6),
    FP16 uniform[-1, 1] operands (ld rounded up to 8), alpha = 1, beta = 0, run
    as HIP graphs; F16 and the refined modes (head and residual planes of the
    same shapes).  The first few dozen launches over fresh operands run up to
    1.3x slower, so each plan is warmed with 60 launches before 20 timed ones."""
    import torch

    import paper_1803_04014_amd as mfg
    import workloads

    dims = workloads.loguniform_dims(6, 4096, 16, 512)
    out = {}
    for mode in ("f16", "refine_a", "split3", "split4"):
        two_a, two_b = mode != "f16", mode in ("split3", "split4")
        probs = []
        for (m_, n_, k_) in dims:
            lda, ldb = -(-int(k_) // 8) * 8, -(-int(n_) // 8) * 8
            a = torch.empty(((2 if two_a else 1) * m_, lda), dtype=torch.float16, device=dev).uniform_(-1, 1)
            b = torch.empty(((2 if two_b else 1) * k_, ldb), dtype=torch.float16, device=dev).uniform_(-1, 1)
            probs.append((a[:m_, :k_], b[:k_, :n_], torch.empty((m_, n_), dtype=torch.float32, device=dev)))
        plan = mfg.GroupedPlan(probs, mode)
        info = plan.info()
        ms = timed(lambda: plan.graph_launch(1.0, 0.0), 20, warm=60)
        key = "grouped_4096" if mode == "f16" else f"grouped_4096_{mode}"
        out[key] = {"gemm_per_s": round(4096 / ms * 1e3, 1), "useful_tflops": round(info["flops"] / ms / 1e9, 2),
                    "hbm_gbs": round(info["bytes"] / ms / 1e6, 1),
                    "pct_hbm": round(100 * info["bytes"] / ms / 1e6 / HBM_GBS, 1), "us": round(ms * 1e3, 1),
                    "work_items": info["work_items"]}
        plan.close()
        del probs
    # from FP32 operands: the plan converts (Eq. R split) every problem in one
    # launch, then runs the grouped kernel; one graph replay holds both
    probs = []
    for (m_, n_, k_) in dims:
        m_, n_, k_ = int(m_), int(n_), int(k_)
        a = torch.empty((m_, -(-k_ // 4) * 4), dtype=torch.float32, device=dev).uniform_(-1, 1)[:, :k_]
        b = torch.empty((k_, -(-n_ // 4) * 4), dtype=torch.float32, device=dev).uniform_(-1, 1)[:, :n_]
        probs.append((a, b, torch.empty((m_, n_), dtype=torch.float32, device=dev)))
    plan = mfg.GroupedPlan(probs, "split3", fp32_in=True)
    info = plan.info()
    ms = timed(lambda: plan.graph_launch(1.0, 0.0), 20, warm=60)
    out["grouped_4096_split3_fp32_in"] = {"gemm_per_s": round(4096 / ms * 1e3, 1),
                                          "useful_tflops": round(info["flops"] / ms / 1e9, 2),
                                          "hbm_gbs": round(info["bytes"] / ms / 1e6, 1),
                                          "pct_hbm": round(100 * info["bytes"] / ms / 1e6 / HBM_GBS, 1),
                                          "us": round(ms * 1e3, 1)}
    plan.close()
    del probs
    return out


def _csv_rows(d: str, suffix: str):
    import csv
    import glob

    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def _per_dispatch(d: str, counter: str, name_part: str) -> float:
    """Mean of `counter` over the dispatches whose kernel name contains name_part."""
    vals = [float(r["Counter_Value"]) for r in _csv_rows(d, "counter_collection.csv")
            if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {name_part!r} under {d}")
    return sum(vals) / len(vals)


def pmc_summarize(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, n) -> int:
    """HBM bytes per launch of the headline GEMM kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for a plain copy of copy_bytes (torch's elementwise copy)."""
    kern = "gemm16_"  # the headline run launches one GEMM kernel
    copy = "copy"
    f_k = _per_dispatch(fetch_dir, "FETCH_SIZE", kern)
    w_k = _per_dispatch(write_dir, "WRITE_SIZE", kern)
    f_c = _per_dispatch(copy_fetch_dir, "FETCH_SIZE", copy)
    w_c = _per_dispatch(copy_write_dir, "WRITE_SIZE", copy)
    f_scale, w_scale = copy_bytes / (f_c * 1024.0), copy_bytes / (w_c * 1024.0)
    fetch, write = f_k * 1024.0 * f_scale, w_k * 1024.0 * w_scale
    algo = 2 * n * n * 2 + 2 * n * n * 4   # A, B in FP16 once; C read and written in FP32
    out = {"kernel_hash": kernel_hash(), "n": n, "kernel_match": kern,
           "fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k,
           "copy_bytes": copy_bytes, "copy_fetch_kib": f_c, "copy_write_kib": w_c,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "hbm_bytes_per_launch": fetch + write, "algorithmic_bytes_per_launch": algo,
           "traffic_over_algorithmic": (fetch + write) / algo}
    with open(PMC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
    return 0


XCDS = 8            # GRBM_GUI_ACTIVE is summed over the XCDs' graphics blocks
SIMDS = 1024        # 256 CUs x 4 SIMDs
MFMA_CYCLES = {"v_mfma_f32_32x32x16": 32}   # SQ_VALU_MFMA_BUSY_CYCLES per instruction (measured: 2^30 / 2^25)


def mfma_summary(d: str, name_part: str) -> int:
    """Markdown rows of MFMA utilisation per dispatch of the kernels whose name
    contains name_part, from one rocprofv3 --pmc run with --kernel-trace:
    SQ_VALU_MFMA_BUSY_CYCLES (summed over the 1024 SIMDs), GRBM_GUI_ACTIVE
    (summed over the 8 XCDs, in shader-clock cycles) and the dispatch's time.
    clock = GUI_ACTIVE / 8 / time; utilisation = busy / (GUI_ACTIVE / 8 * 1024)
    (rocprofv3's MfmaUtil uses the largest XCD's GUI_ACTIVE instead of the mean);
    MOPS counters (per 512 flops) give the matrix flops and the rate."""
    import collections

    per = collections.defaultdict(dict)
    for r in _csv_rows(d, "counter_collection.csv"):
        if name_part not in r["Kernel_Name"]:
            continue
        k = int(r["Dispatch_Id"])
        per[k][r["Counter_Name"]] = float(r["Counter_Value"])
        per[k]["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per[k]["name"] = r["Kernel_Name"].split("(")[0]
    if not per:
        raise SystemExit(f"no dispatches of kernels matching {name_part!r} under {d}")
    print("| dispatch | kernel | time us | MFMA busy cycles | GUI_ACTIVE / 8 | clock GHz | MFMA util | matrix TFLOP/s |")
    print("|---|---|---|---|---|---|---|---|")
    for k, v in sorted(per.items()):
        gui = v.get("GRBM_GUI_ACTIVE", 0.0) / XCDS
        busy = v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        mops = sum(x for c, x in v.items() if c.startswith("SQ_INSTS_VALU_MFMA_MOPS"))
        clk = gui / v["ns"] if gui else 0.0
        util = busy / (gui * SIMDS) if gui else 0.0
        tf = mops * 512 / v["ns"] / 1e3 if mops else 0.0
        print(f"| {k} | `{v['name']}` | {v['ns'] / 1e3:.1f} | {busy:.4g} | {gui:.4g} | {clk:.3f} | {util:.3f} | "
              f"{tf:.1f} |")
    return 0


def counter_table(d: str, name_part: str) -> int:
    """Markdown table of every counter of a rocprofv3 --pmc output folder, mean
    over the dispatches of the kernels whose name contains name_part (the
    first dispatch, a warm-up at a cold clock, left out when there are
    others), with the SQ_WAIT_* and SQ_ACTIVE_* counters (wave-level, in the
    same units as SQ_WAVE_CYCLES) also as a share of SQ_WAVE_CYCLES when that
    counter was collected."""
    import collections

    per = collections.defaultdict(dict)
    for r in _csv_rows(d, "counter_collection.csv"):
        if name_part not in r["Kernel_Name"]:
            continue
        k = int(r["Dispatch_Id"])
        per[k][r["Counter_Name"]] = float(r["Counter_Value"])
        per[k]["time_ns"] = float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    if not per:
        raise SystemExit(f"no dispatches of kernels matching {name_part!r} under {d}")
    keys = sorted(per)
    if len(keys) > 1:
        keys = keys[1:]
    names = sorted({c for k in keys for c in per[k]})
    mean = {c: sum(per[k].get(c, 0.0) for k in keys) / len(keys) for c in names}
    wave = mean.get("SQ_WAVE_CYCLES")
    print(f"dispatches averaged: {len(keys)} ({keys[0]}..{keys[-1]})")
    print("| counter | mean per dispatch | share of SQ_WAVE_CYCLES |")
    print("|---|---|---|")
    for c in names:
        share = f"{mean[c] / wave:.3f}" if wave and c.startswith(("SQ_WAIT", "SQ_ACTIVE")) else ""
        print(f"| {c} | {mean[c]:.6g} | {share} |")
    return 0


def trace_overlap(d: str, name_part: str = "mfg::") -> int:
    """From a rocprofv3 --kernel-trace output folder: how the kernels whose name
    contains name_part overlapped in time across HIP streams -- kernels per
    stream, the largest number running at once, and the share of the busy
    time with kernels of two or more streams on the device."""
    rows = [r for r in _csv_rows(d, "kernel_trace.csv") if name_part in r["Kernel_Name"]]
    if not rows:
        raise SystemExit(f"no kernels matching {name_part!r} under {d}")
    ev, per_stream = [], {}
    for r in rows:
        s, e, q = int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Stream_Id") or r.get("Queue_Id")
        per_stream[q] = per_stream.get(q, 0) + 1
        ev += [(s, 1, q), (e, -1, q)]
    ev.sort()
    active, by_q, most, busy, multi, last = 0, {}, 0, 0, 0, ev[0][0]
    for t, dlt, q in ev:
        span = t - last
        if active > 0:
            busy += span
        if sum(1 for v in by_q.values() if v > 0) >= 2:
            multi += span
        last = t
        active += dlt
        by_q[q] = by_q.get(q, 0) + dlt
        most = max(most, active)
    out = {"kernels": len(rows), "kernels_per_stream": per_stream, "max_concurrent_kernels": most,
           "busy_ms": round(busy / 1e6, 3), "share_of_busy_time_with_two_or_more_streams": round(multi / max(busy, 1), 3)}
    print(json.dumps(out))
    return 0


def copy_probe(nbytes: int) -> int:
    """A plain device copy of nbytes, three times: the calibration kernel for
    the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {nbytes} bytes x 3", flush=True)
    return 0


def fused_legs(dev, sizes=(2048, 4096, 8192), reps: int = 8) -> dict:
    """The refined modes from FP32 operands two ways, timed interleaved: the
    default two-pass path (split pass into workspace planes, then the GEMM on
    them) and the fused kernel that splits while staging its tiles (the last
    configuration of the mode, no workspace).  Per mode and N: milliseconds
    (median of per-launch times) and useful TFLOP/s."""
    import torch

    import paper_1803_04014_amd as mfg

    out = {}
    for n in sizes:
        gen = torch.Generator(device=dev)
        gen.manual_seed(n)
        A = torch.randn((n, n), device=dev, generator=gen)
        B = torch.randn((n, n), device=dev, generator=gen)
        C = torch.zeros((n, n), device=dev)
        fl = 2.0 * n ** 3
        for mode in ("split3", "refine_a", "bf16_split3"):
            fused = mfg.num_configs(mode) - 1
            assert mfg.config_name(mode, fused).startswith("fused")
            t = {"two_pass": [], "fused": []}
            for _ in range(3):
                t["two_pass"] += launch_times(lambda: mfg.gemm(A, B, C, 1.0, 0.0, mode=mode), reps, warm=2)
                t["fused"] += launch_times(lambda: mfg.gemm(A, B, C, 1.0, 0.0, mode=mode, config=fused), reps, warm=2)
            e = {}
            for k, v in t.items():
                st = rate_stats(fl, v)
                e[k] = {"ms": round(fl / st["tflops_median"] / 1e9, 4), "tflops": st["tflops_median"]}
            e["fused_over_two_pass"] = round(e["fused"]["ms"] / e["two_pass"]["ms"], 3)
            out[f"{mode}_n{n}"] = e
        del A, B, C
    return out


def solve_legs(dev, sizes=(2048, 8192), modes=("f32", "split3", "f16")) -> dict:
    """The iterative-refinement solver on the GEMM (mfg_solve_ir): FP64 A of
    condition ~1e3 (Q1 diag(s) Q2^T, s log-spaced; n = 2048) or normal(0, 1)
    plus sqrt(n) I (n = 8192: orthogonal factors of that size take minutes on
    the host), one normal right-hand side, tolerance 2^-50; per mode the
    wall time of one solve (after one untimed), of the LU alone, the
    corrections made and the final backward error."""
    import torch

    import paper_1803_04014_amd as mfg
    import workloads

    out = {}
    for n in sizes:
        if n <= 2048:
            A = torch.from_numpy(workloads.conditioned(5, n, 1e3)).to(dev)
        else:
            gen = torch.Generator(device=dev)
            gen.manual_seed(n)
            A = torch.randn((n, n), dtype=torch.float64, device=dev, generator=gen)
            A += n ** 0.5 * torch.eye(n, dtype=torch.float64, device=dev)
        B = torch.randn((n, 1), dtype=torch.float64, device=dev)
        for mode in modes:
            X = torch.zeros((n, 1), dtype=torch.float64, device=dev)
            mfg.solve_ir(A, B, X, mode=mode, max_iter=30)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = mfg.solve_ir(A, B, X, mode=mode, max_iter=30)
            t1 = time.perf_counter()
            a32 = A.float()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            mfg.lu_factor(a32, mode)
            t3 = time.perf_counter()
            out[f"{mode}_n{n}"] = {"solve_ms": round((t1 - t0) * 1e3, 1), "lu_ms": round((t3 - t2) * 1e3, 1),
                                   "corrections": r["iters"], "backward_error": r["berr"]}
            del a32
        del A, B
    return out


def kernel_only(mode: str, n: int, steps: int, warmup: int) -> int:
    """`steps` launches of one mode's GEMM at n^3 on operands already in the
    mode's preconverted form (C = A B + C, alpha = beta = 1): the run the MFMA
    counter passes profile.  Prints the kernel's average time and rate."""
    import torch

    import paper_1803_04014_amd as mfg

    dev = "cuda:0"
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    A32 = torch.rand((n, n), device=dev, generator=g) * 2 - 1
    B32 = torch.rand((n, n), device=dev, generator=g) * 2 - 1
    C = torch.rand((n, n), device=dev, generator=g) * 2 - 1
    if mode == "f32":
        pa, pb = A32, B32
    else:
        ld = n
        nb = mfg.convert_bytes(n, n, ld, mode)
        bufa = torch.empty(nb, dtype=torch.uint8, device=dev)
        bufb = torch.empty(nb, dtype=torch.uint8, device=dev)
        mfg.convert(A32, bufa, ld, mode)
        mfg.convert(B32, bufb, ld, mode)
        if mode == "fp8":
            pa, pb = bufa[:n * ld].view(n, ld), bufb[:n * ld].view(n, ld)
        else:
            pa = bufa.view(torch.float16).view(-1, ld)
            pb = bufb.view(torch.float16).view(-1, ld)
    run = lambda: mfg.gemm(pa, pb, C, 1.0, 1.0, mode=mode, preconverted=True, M=n, K=n)
    ms = timed(run, steps, warm=warmup)
    products = {"refine_a": 2, "split3": 3, "split4": 4, "bf16_split3": 3}.get(mode, 1)
    fl = 2.0 * n ** 3
    print(json.dumps({"kernel_only": mode, "n": n, "ms": round(ms, 4), "useful_tflops": round(fl / ms / 1e9, 1),
                      "executed_tflops": round(products * fl / ms / 1e9, 1)}), flush=True)
    return 0


def mfma_ceiling(dev, iters: int = 2048, workgroups_per_cu: int = 2) -> dict:
    """Register-only MFMA loops (mfg_probe_mfma) on random and on all-zero
    operands: both FP16 MFMA shapes (uniform[-1, 1] values) and the FP8 E4M3
    32x32x64 instruction (uniform[-1, 1] rounded to E4M3): the matrix-core rate
    the chip sustains with no memory traffic, i.e. the ceiling the GEMM kernels
    work against."""
    import ctypes

    import torch

    import paper_1803_04014_amd as mfg

    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    wg = ncu * workgroups_per_cu
    rnd = torch.empty(8192, dtype=torch.float16, device=dev).uniform_(-1, 1)
    zero = torch.zeros(8192, dtype=torch.float16, device=dev)
    rnd8 = torch.empty(16384, dtype=torch.float32, device=dev).uniform_(-1, 1).to(torch.float8_e4m3fn).view(torch.uint8)
    zero8 = torch.zeros(16384, dtype=torch.uint8, device=dev)
    out = torch.empty(wg * 256, dtype=torch.float32, device=dev)
    res = {}
    for shape, sname, ops_r, ops_z in ((0, "32x32x16", rnd, zero), (1, "16x16x32", rnd, zero),
                                       (2, "32x32x64_e4m3", rnd8, zero8)):
        for ops, oname in ((ops_r, "random"), (ops_z, "zero")):
            fl = ctypes.c_double()

            def launch():
                mfg.capi.check("mfg_probe_mfma", mfg.lib().mfg_probe_mfma(
                    shape, ctypes.c_void_p(ops.data_ptr()), wg, iters, ctypes.c_void_p(out.data_ptr()),
                    ctypes.byref(fl), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
            ms = timed(launch, 5, warm=2)
            res[f"{sname}_{oname}"] = {"tflops": round(fl.value / ms / 1e9, 1), "ms": round(ms, 3)}
    res["workgroups"] = wg
    res["waves_per_simd"] = workgroups_per_cu
    return res


def served_errors(trace, views, per_mode: int = 3, rows: int = 16):
    """Part of the CPU oracle leg: max relative error vs FP64 of a few served
    requests per mode, the first `per_mode` of each mode whatever their size,
    on `rows` sampled rows of each (the oracle computes their exact products)."""
    import numpy as np

    import oracle

    errs = {}
    for mode in sorted({r["mode"] for r in trace}):
        picked = [i for i, r in enumerate(trace) if r["mode"] == mode][:per_mode]
        worst, shapes = 0.0, []
        for i in picked:
            a, b, c = views[i]
            M = a.shape[0]
            rsel = oracle.sample_rows(M, n=rows, seed=i)
            A = a.cpu().numpy()
            B = b.cpu().numpy()
            ref = oracle.exact(A, B, 1.0, 0.0, None, rows=rsel)
            got = c.cpu().numpy().astype(np.float64)[rsel]
            err = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
            worst = max(worst, float(err))
            shapes.append(f"{M}x{b.shape[1]}x{a.shape[1]}")
        errs[mode] = {"max_rel": worst, "sampled": shapes, "rows_per_request": rows}
    return errs


def serving_leg(rate: float, seconds: float, max_requests: int, seed: int, pools, budget: float = 200e9,
                slots: int = 4, max_group: int = 16):
    """Replay a Poisson trace of GEMM requests (M, N, K log-uniform in [32, 4096],
    modes F16 / BF16 / SPLIT3 / FP8, operands sub-blocks of resident 4096 x 4096
    FP32 pools, a distinct C per request, alpha = 1, beta = 0) into mfg_server:
    min(max_requests, rate * seconds) requests.  Latency = completion observed -
    submit, per request."""
    import numpy as np
    import torch

    import paper_1803_04014_amd as mfg
    import workloads

    dA, dB = pools
    n = max(1, min(max_requests, int(rate * seconds)))
    trace = workloads.serving_trace(seed, rate, n)
    sizes = [r["M"] * r["N"] for r in trace]
    arena = torch.empty(int(sum(sizes)), dtype=torch.float32, device=dA.device)
    views, off = [], 0
    for r, sz in zip(trace, sizes):
        (ar, ac), (br, bc) = r["a_off"], r["b_off"]
        views.append((dA[ar:ar + r["M"], ac:ac + r["K"]], dB[br:br + r["K"], bc:bc + r["N"]],
                      arena[off:off + sz].view(r["M"], r["N"])))
        off += sz
    torch.cuda.synchronize()
    server = mfg.Server(int(budget), slots=slots, max_group=max_group)
    tickets = []
    t0 = time.perf_counter()
    for r, (a, b, c) in zip(trace, views):
        while time.perf_counter() - t0 < r["t"]:
            pass
        tickets.append(server.submit(a, b, c, r["mode"], 1.0, 0.0))
    server.drain()
    polled = [server.poll(t) for t in tickets]
    stats = server.stats()
    server.close()
    res = [x[1] for x in polled]
    lat = np.array([(x["t_end_ns"] - x["t_submit_ns"]) * 1e-6 for x in res])
    wait = np.array([(x["t_start_ns"] - x["t_submit_ns"]) * 1e-6 for x in res])  # queued until launched
    big = np.array([x["flops"] for x in res])
    span = (max(x["t_end_ns"] for x in res) - min(x["t_submit_ns"] for x in res)) * 1e-9
    flops = sum(x["flops"] for x in res)
    tail = lat >= np.percentile(lat, 99)
    out = {"rate_per_s": rate, "requests": n, "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
           "p50_wait_ms": round(float(np.percentile(wait, 50)), 3),
           "p99_wait_ms": round(float(np.percentile(wait, 99)), 3),
           "slowest_1pct_mean_gflop": round(float(big[tail].mean()) / 1e9, 2),
           "useful_tflops": round(flops / span / 1e12, 2), "offered_tflops": round(flops / trace[-1]["t"] / 1e12, 2),
           "launches": stats["launches"], "mean_group": round(float(np.mean([x["group_size"] for x in res])), 2),
           "max_concurrent_slots": stats["max_concurrent_slots"], "slots": slots,
           "failed": stats["failed"] + sum(1 for st, _ in polled if st != 0),
           "peak_converted_gb": round(stats["peak_bytes_in_use"] / 1e9, 3)}
    return out, trace, views


def rate_stats(flops: float, ms: list) -> dict:
    """Per-launch rates of `flops` over launch times `ms`: the harmonic mean
    (flops over the mean time, the paper's convention), median, p10 and p90."""
    import numpy as np

    t = np.asarray(ms, dtype=np.float64)
    r = flops / (t * 1e-3) / 1e12
    return {"tflops_hmean": round(flops / (t.mean() * 1e-3) / 1e12, 2), "tflops_median": round(float(np.median(r)), 2),
            "tflops_p10": round(float(np.percentile(r, 10)), 2), "tflops_p90": round(float(np.percentile(r, 90)), 2),
            "launches": int(t.size)}


def launch_times(fn, reps: int, warm: int = 2) -> list:
    """Per-launch milliseconds of fn() (HIP events around each launch on the current stream)."""
    import torch

    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def smi_sample():
    """One amd-smi reading of the graphics clocks (MHz, per XCD) and socket power (W), or None."""
    import subprocess

    try:
        out = subprocess.run(["amd-smi", "metric", "-g", "0", "-c", "-p", "--json"], capture_output=True, text=True,
                             timeout=10).stdout
        d = json.loads(out)
        g = d["gpu_data"][0] if isinstance(d, dict) and "gpu_data" in d else (d[0] if isinstance(d, list) else d)
        clk = [v["clk"]["value"] for k, v in g["clock"].items()
               if k.startswith("gfx_") and isinstance(v, dict) and isinstance(v.get("clk"), dict)]
        pw = g["power"]["socket_power"]["value"]
        return {"sclk_mhz": [float(c) for c in clk], "power_w": float(pw)}
    except Exception:
        return None


def sustained_clock(step, flops: float, seconds: float) -> dict:
    """Run `step` back to back for `seconds` while another thread samples the
    graphics clocks and socket power: the clock the headline kernel runs at
    under a sustained load (the dense peak assumes 2.4 GHz)."""
    import threading

    import torch

    samples, stop = [], [False]

    def sampler():
        while not stop[0]:
            ts = time.perf_counter()
            x = smi_sample()
            if x is None:
                return
            samples.append((ts, time.perf_counter(), x))
            time.sleep(0.05)

    th = threading.Thread(target=sampler, daemon=True)
    for _ in range(20):
        step()
    torch.cuda.synchronize()
    th.start()
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            step()
        torch.cuda.synchronize()
        k += 20
    el = time.perf_counter() - t0
    stop[0] = True
    th.join(timeout=15)
    out = {"seconds": round(el, 2), "launches": k, "tflops": round(flops * k / el / 1e12, 1)}
    # readings taken wholly inside the loaded interval, past its first quarter
    mid = [x for (a, b, x) in samples if a >= t0 + 0.25 * el and b <= t0 + el]
    if mid:
        clks = sorted(c for s_ in mid for c in s_["sclk_mhz"])
        out.update({"sclk_mhz_mean": round(sum(clks) / len(clks), 1), "sclk_mhz_median": clks[len(clks) // 2],
                    "sclk_mhz_min": clks[0], "sclk_mhz_max": clks[-1],
                    "power_w_mean": round(sum(s_["power_w"] for s_ in mid) / len(mid), 1), "samples": len(mid)})
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_single_thread(n: int = 1024) -> dict:
    """The FP64 oracle GEMM at n^3 on one host thread (a child process with
    OMP_NUM_THREADS=1): context for the many-core cpu_baseline."""
    import subprocess

    code = ("import time, sys; sys.path.insert(0, %r); import numpy as np, oracle, workloads; "
            "A, B = workloads.uniform(2, [(%d, %d), (%d, %d)]); oracle.exact(A[:8], B); "
            "t = time.perf_counter(); oracle.exact(A, B); dt = time.perf_counter() - t; "
            "print(dt, oracle.num_threads())") % (ROOT, n, n, n, n)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    dt, thr = r.stdout.split()[-2:]
    return {"n": n, "seconds": round(float(dt), 3), "gflops": round(2.0 * n ** 3 / float(dt) / 1e9, 2),
            "threads": int(thr)}


def precision_legs(dev, cpu: bool) -> dict:
    """The refinement study (paper Sec. VII.B) on FP32 inputs drawn two ways,
    normal(0, 1) (seed 3) and sign * 2^u with u uniform in [-10, 10] (seed 4),
    at N = 4096 and 8192: for each mode, the end-to-end time from FP32
    operands (conversion included) and, with the oracle, the max and
    Frobenius errors relative to the exact FP64 product on 32 sampled rows
    (reduced in FP64 on the GPU)."""
    import numpy as np
    import torch

    import paper_1803_04014_amd as mfg
    import workloads

    modes = ("f16", "refine_a", "split3", "split4", "f32", "bf16", "bf16_split3", "bf16_split6")
    products = {"refine_a": 2, "split3": 3, "split4": 4, "bf16_split3": 3, "bf16_split6": 6}
    out = {}
    for dist, seed in (("normal", 3), ("pow2", 4)):
        for n in (4096, 8192):
            A, B = workloads.by_name(dist, seed, [(n, n), (n, n)])
            dA, dB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
            dC = torch.empty((n, n), dtype=torch.float32, device=dev)
            fl = 2.0 * n ** 3
            ref = rows = None
            if cpu:
                import oracle

                rows = oracle.sample_rows(n, n=32, seed=seed)
                ref = torch.from_numpy(oracle.exact(A, B, 1.0, 0.0, None, rows=rows)).to(dev)
                ridx = torch.from_numpy(rows).to(dev)
            row = {}
            for mode in modes:
                ms = launch_times(lambda: mfg.gemm(dA, dB, dC, 1.0, 0.0, mode=mode), 3, warm=1)
                st = rate_stats(fl, ms)
                e = {"useful_tflops": st["tflops_hmean"],
                     "executed_tflops": round(products.get(mode, 1) * st["tflops_hmean"], 1),
                     "ms": round(float(np.mean(ms)), 3)}
                if cpu:
                    sub = dC.index_select(0, ridx).contiguous()
                    o4 = torch.zeros(4, dtype=torch.float64, device=dev)
                    mfg.error_norms(sub, ref, o4)
                    o = o4.cpu().numpy()
                    e["max_rel"], e["fro_rel"] = float(o[0] / o[3]), float(o[1] / o[2])
                row[mode] = e
            out[f"{dist}_n{n}"] = row
            del dA, dB, dC
    return out


def grouped_problem_set(dev, mode: str, seed: int = 6, count: int = 4096, lo: int = 16, hi: int = 512):
    """The grouped workload: `count` problems with M, N, K log-uniform in [lo, hi]
    (seed), FP16 uniform[-1, 1] operands in the mode's preconverted form (ld
    rounded up to 8; head and residual planes for the refined modes), FP32 C."""
    import torch

    import workloads

    two_a, two_b = mode != "f16", mode in ("split3", "split4")
    probs = []
    for (m_, n_, k_) in workloads.loguniform_dims(seed, count, lo, hi):
        m_, n_, k_ = int(m_), int(n_), int(k_)
        lda, ldb = -(-k_ // 8) * 8, -(-n_ // 8) * 8
        a = torch.empty(((2 if two_a else 1) * m_, lda), dtype=torch.float16, device=dev).uniform_(-1, 1)
        b = torch.empty(((2 if two_b else 1) * k_, ldb), dtype=torch.float16, device=dev).uniform_(-1, 1)
        probs.append((a[:m_, :k_], b[:k_, :n_], torch.empty((m_, n_), dtype=torch.float32, device=dev)))
    return probs


def grouped_autotune_leg(dev) -> dict:
    """The grouped tile-class tuner on the 4096-problem mix of F16 and SPLIT3
    (it records the fastest class for every size bucket of the mix), then the
    default plan against the one built after tuning: when they launch the same
    classes there is one timing and no gain, else both are timed interleaved
    as HIP graph replays after the same warm-up."""
    import numpy as np

    import paper_1803_04014_amd as mfg

    out = {}
    for mode in ("f16", "split3"):
        mfg.lib().mfg_tune_clear()
        probs = grouped_problem_set(dev, mode)
        default = mfg.GroupedPlan(probs, mode)
        best, tms = mfg.grouped_autotune(probs, mode, reps=5)
        tuned = mfg.GroupedPlan(probs, mode)
        e = {"classes": mfg.grouped_tile_classes(mode), "default_plan": {str(k): v for k, v in default.classes().items()},
             "tuner_best": best, "tuner_us": round(tms * 1e3, 1),
             "tuned_plan": {str(k): v for k, v in tuned.classes().items()}}
        run_d, run_t = (lambda: default.graph_launch(1.0, 0.0)), (lambda: tuned.graph_launch(1.0, 0.0))
        if default.classes() == tuned.classes():
            e.update({"same_as_default": True, "us": round(float(np.median(launch_times(run_d, 20, warm=60))) * 1e3, 1)})
        else:
            td, tt = launch_times(run_d, 5, warm=60), launch_times(run_t, 5, warm=60)
            for _ in range(3):
                td += launch_times(run_d, 5, warm=5)
                tt += launch_times(run_t, 5, warm=5)
            e.update({"same_as_default": False, "default_us": round(float(np.median(td)) * 1e3, 1),
                      "tuned_us": round(float(np.median(tt)) * 1e3, 1)})
        out[mode] = e
        default.close()
        tuned.close()
        del probs
    mfg.lib().mfg_tune_clear()
    return out


def write_tune_table(path: str) -> int:
    """Tune and save the table shipped with the library (MFG_TUNE_TABLE): the
    GEMM configuration for F16 (preconverted) at 4096^3, 8192 x 2048 x 4096,
    2048 x 2048 x 8192 and 1536^3, and for SPLIT3 and REFINE_A from FP32 at
    2048^3 and 4096^3 (the two-pass configurations against the fused kernel);
    the grouped tile class for the F16 and SPLIT3 4096-problem mixes."""
    import torch

    import paper_1803_04014_amd as mfg

    dev = torch.device("cuda", 0)
    mfg.lib().mfg_tune_clear()
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    A32 = torch.rand((8192, 8192), device=dev, generator=gen) * 2 - 1
    B32 = torch.rand((8192, 8192), device=dev, generator=gen) * 2 - 1
    A16, B16 = A32.half(), B32.half()
    rows = []
    for (m_, n_, k_) in ((4096, 4096, 4096), (8192, 2048, 4096), (2048, 2048, 8192), (1536, 1536, 1536)):
        a, b = A16[:m_, :k_].contiguous(), B16[:k_, :n_].contiguous()
        c = torch.empty((m_, n_), dtype=torch.float32, device=dev)
        best, ms = mfg.autotune(a, b, c, "f16", reps=3, preconverted=True)
        rows.append({"mode": "f16", "shape": [m_, n_, k_], "config": mfg.config_name("f16", best), "ms": round(ms, 4)})
    for mode in ("split3", "refine_a"):
        for n in (2048, 4096):
            a, b = A32[:n, :n].contiguous(), B32[:n, :n].contiguous()
            c = torch.empty((n, n), dtype=torch.float32, device=dev)
            best, ms = mfg.autotune(a, b, c, mode, reps=3)
            rows.append({"mode": mode, "shape": [n, n, n], "config": mfg.config_name(mode, best), "ms": round(ms, 4)})
    del A32, B32, A16, B16
    for mode in ("f16", "split3"):
        probs = grouped_problem_set(dev, mode)
        best, ms = mfg.grouped_autotune(probs, mode, reps=5)
        rows.append({"mode": mode, "grouped_4096_tile": best, "us": round(ms * 1e3, 1)})
        del probs
    st = mfg.lib().mfg_tune_save(path.encode())
    print(json.dumps({"tune_table": path, "status": st, "entries": rows}), flush=True)
    mfg.lib().mfg_tune_clear()
    return 0 if st == 0 else 1


def autotune_leg(dA, dB, dev) -> dict:
    """The autotuner on a few FP16 shapes: the default configuration against the
    tuned one, timed interleaved (default, tuned, default, ...) after the same
    warm-up; when the tuner keeps the default there is one timing and no gain."""
    import numpy as np
    import torch

    import paper_1803_04014_amd as mfg

    out = {}
    mfg.lib().mfg_tune_clear()
    for (m_, n_, k_) in ((4096, 4096, 4096), (8192, 2048, 4096), (2048, 2048, 8192), (1536, 1536, 1536)):
        a = dA[:m_, :k_].contiguous()
        b = dB[:k_, :n_].contiguous()
        c = torch.empty((m_, n_), dtype=torch.float32, device=dev)
        m16 = mfg.MFG_F16 | mfg.MFG_IN_PRECONVERTED
        default = mfg.lib().mfg_tune_lookup(m_, n_, k_, m16)
        best, _ = mfg.autotune(a, b, c, "f16", reps=3, preconverted=True)
        fl = 2.0 * m_ * n_ * k_
        run = lambda cfg: mfg.gemm(a, b, c, 1.0, 0.0, mode="f16", preconverted=True, config=cfg)
        e = {"default_config": mfg.config_name("f16", default), "tuned_config": mfg.config_name("f16", best)}
        if best == default:
            ms = launch_times(lambda: run(default), 10, warm=5)
            e.update({"same_as_default": True, "tflops": rate_stats(fl, ms)["tflops_median"]})
        else:
            td, tt = [], []
            for _ in range(3):
                td += launch_times(lambda: run(default), 5, warm=3)
                tt += launch_times(lambda: run(best), 5, warm=3)
            e.update({"same_as_default": False, "default_tflops": rate_stats(fl, td)["tflops_median"],
                      "tuned_tflops": rate_stats(fl, tt)["tflops_median"]})
        out[f"{m_}x{n_}x{k_}"] = e
    mfg.lib().mfg_tune_clear()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target oracle time for cpu_baseline")
    ap.add_argument("--sclk-seconds", type=float, default=2.0, help="sustained-load clock sampling")
    ap.add_argument("--serve-seconds", type=float, default=8.0, help="per arrival rate (at most 20000 requests)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, metavar="BYTES", help="only run the counter-calibration copy")
    ap.add_argument("--pmc-summarize", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="only turn four rocprofv3 --pmc output folders into the traffic record")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--grouped-only", action="store_true", help="only the grouped-plan legs (one JSON line)")
    ap.add_argument("--write-tune-table", metavar="PATH", help="only tune and save the shipped tuned table")
    ap.add_argument("--solve-only", action="store_true", help="only the iterative-refinement solve legs")
    ap.add_argument("--fused-only", action="store_true",
                    help="only the refined modes from FP32: two-pass against the fused kernel (one JSON line)")
    ap.add_argument("--serving-only", action="store_true", help="only the serving legs (one JSON line)")
    ap.add_argument("--kernel-only", metavar="MODE", help="only time MODE's GEMM at N^3 on preconverted operands")
    ap.add_argument("--mfma-ceiling", action="store_true", help="only the register-only MFMA ceiling probe")
    ap.add_argument("--mfma-summary", nargs=2, metavar=("DIR", "KERNEL"),
                    help="only print MFMA utilisation per dispatch from a rocprofv3 --pmc output folder")
    ap.add_argument("--counter-table", nargs=2, metavar=("DIR", "KERNEL"),
                    help="only print every counter's mean per dispatch from a rocprofv3 --pmc output folder")
    ap.add_argument("--trace-overlap", metavar="DIR",
                    help="only print how the library's kernels overlapped across streams in a kernel trace")
    args = ap.parse_args()
    if args.trace_overlap:
        return trace_overlap(args.trace_overlap)
    if args.mfma_summary:
        return mfma_summary(*args.mfma_summary)
    if args.counter_table:
        return counter_table(*args.counter_table)
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.pmc_summarize:
        return pmc_summarize(*args.pmc_summarize, args.copy_bytes, args.n)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (no multi-GPU path)",
              file=sys.stderr)
        return 2
    if args.kernel_only:
        return kernel_only(args.kernel_only, args.n, args.steps, args.warmup)
    if args.mfma_ceiling:
        import torch

        print(json.dumps({"mfma_ceiling": mfma_ceiling(torch.device("cuda", 0))}), flush=True)
        return 0
    if args.grouped_only:
        import torch

        print(json.dumps(grouped_legs(timed, torch.device("cuda", 0))), flush=True)
        return 0
    if args.write_tune_table:
        return write_tune_table(args.write_tune_table)
    if args.solve_only:
        import torch

        print(json.dumps({"solve_ir": solve_legs(torch.device("cuda", 0))}), flush=True)
        return 0
    if args.fused_only:
        import torch

        print(json.dumps({"fused_fp32_in": fused_legs(torch.device("cuda", 0))}), flush=True)
        return 0

    import numpy as np
    import torch

    import paper_1803_04014_amd as mfg
    import workloads

    dev = "cuda:0"
    torch.cuda.set_device(0)

    def serving_legs(rates, cpu):
        gen = torch.Generator(device=dev)
        gen.manual_seed(7)
        pools = (torch.randn((4096, 4096), device=dev, generator=gen),
                 torch.randn((4096, 4096), device=dev, generator=gen))
        serving = {}
        for rate in rates:
            log(f"bench: serving at {rate:.0f} requests/s")
            srv, trace, views = serving_leg(rate, args.serve_seconds, 20000, 7, pools)
            if cpu:
                srv["errors_vs_fp64"] = served_errors(trace, views)
            serving[f"lambda_{int(rate)}"] = srv
            del views
        return serving

    rates = (200.0, 500.0, 1000.0, 2000.0, 5000.0)
    if args.serving_only:
        print(json.dumps({"serving": serving_legs(rates, not args.no_cpu)}), flush=True)
        return 0

    N = args.n
    log(f"bench: generating inputs N={N}")
    A32, B32, C0 = workloads.uniform(2, [(N, N), (N, N), (N, N)])
    dA32 = torch.from_numpy(A32).to(dev)
    dB32 = torch.from_numpy(B32).to(dev)
    dC0 = torch.from_numpy(C0).to(dev)
    dA = torch.empty((N, N), dtype=torch.float16, device=dev)
    dB = torch.empty((N, N), dtype=torch.float16, device=dev)
    mfg.round_f16(dA32, dA)   # untimed rounding (paper Sec. VI)
    mfg.round_f16(dB32, dB)
    dC = dC0.clone()
    flops = 2.0 * N * N * N

    def step():
        mfg.gemm(dA, dB, dC, 1.0, 1.0, mode="f16", preconverted=True)

    log("bench: warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    log("bench: timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        step()
        evs[i][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    times = [a.elapsed_time(b) for a, b in evs]
    kernel_ms = sum(times) / args.steps
    value = flops * args.steps / wall / 1e12
    achieved = flops / (kernel_ms * 1e-3) / 1e12

    traffic = None
    if os.path.exists(PMC_FILE):
        with open(PMC_FILE) as f:
            pmc = json.load(f)
        if pmc.get("kernel_hash") == kernel_hash() and pmc.get("n") == N:
            traffic = pmc.get("hbm_bytes_per_launch")

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": round(value / PAPER_V100_TFLOPS, 2), "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": f"square GEMM C=A*B+C, M=N=K={N}, FP16 inputs (FP32 uniform[-1,1] rounded, "
                               "untimed), FP32 accumulate and output, alpha=beta=1, row-major",
                   "M": N, "N": N, "K": N, "mode": "f16", "seed": 2},
        "pct_mfma_peak": round(100.0 * value / PEAK_TFLOPS["f16"], 2),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_TFLOPS["f16"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f16"], 4), "traffic": traffic,
                     "kernel_ms": round(kernel_ms, 4), "kernel_hash": kernel_hash()},
        "launch_stats": rate_stats(flops, times),
    }
    log(f"bench: f16 N={N}: {value:.1f} TFLOP/s wall, kernel {kernel_ms:.3f} ms -> {achieved:.1f} TFLOP/s")

    # the clock under a sustained headline load, and the roofline at that clock
    if args.sclk_seconds > 0:
        log("bench: sustained clock")
        sc = sustained_clock(step, flops, args.sclk_seconds)
        out["sustained_clock"] = sc
        if "sclk_mhz_mean" in sc:
            out["roofline"]["frac_at_measured_clock"] = round(
                sc["tflops"] / (PEAK_TFLOPS["f16"] * sc["sclk_mhz_mean"] / 2400.0), 4)

    # fresh result for the error figures: C = A B + C0 once
    results = {}
    dC.copy_(dC0)
    step()
    results["f16"] = dC
    if not args.no_extras:
        dCs = dC0.clone()
        mfg.gemm(dA32, dB32, dCs, 1.0, 1.0, mode="split3")
        results["split3"] = dCs
        dCf = dC0.clone()
        mfg.gemm(dA32, dB32, dCf, 1.0, 1.0, mode="f32")
        results["f32"] = dCf
    torch.cuda.synchronize()

    # ----------------------------------------------------- CPU oracle leg
    if not args.no_cpu:
        import oracle  # the FP64 CPU oracle: only this leg of the benchmark uses it

        # per-row cost from two probes (the difference removes the fixed cost
        # of widening the operands to FP64)
        probe_t = []
        for n_probe in (32, 160):
            rows_probe = np.arange(n_probe, dtype=np.int64) * max(1, N // n_probe)
            t = time.perf_counter()
            oracle.exact(A32, B32, 1.0, 1.0, C0, rows=rows_probe)
            probe_t.append(time.perf_counter() - t)
        per_row = max((probe_t[1] - probe_t[0]) / 128, 1e-6)
        fixed = max(probe_t[0] - 32 * per_row, 0.0)
        nrows = int(max(8, min(N, (args.cpu_seconds - fixed) / per_row)))
        rows = np.unique(np.linspace(0, N - 1, nrows).astype(np.int64))
        log(f"bench: cpu oracle on {len(rows)} rows")
        t = time.perf_counter()
        ref = oracle.exact(A32, B32, 1.0, 1.0, C0, rows=rows)
        cpu_s = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(2.0 * len(rows) * N * N / cpu_s / 1e12, 5), "unit": "TFLOP/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"FP64 GEMM of {len(rows)} of {N} rows (x {N} x {N}), {cpu_s:.1f} s",
                               "cpu_model": cpu_model()}
        # FP64 error reductions on the GPU (rows of C against the oracle's rows)
        dref = torch.from_numpy(ref).to(dev)
        ridx = torch.from_numpy(rows).to(dev)
        errs = {}
        for name, t_c in results.items():
            sub = t_c.index_select(0, ridx).contiguous()
            o4 = torch.zeros(4, dtype=torch.float64, device=dev)
            mfg.error_norms(sub, dref, o4)
            o = o4.cpu().numpy()
            errs[name] = {"max_rel": float(o[0] / o[3]), "fro_rel": float(o[1] / o[2])}
        out["errors_vs_fp64"] = errs
        out["max_rel_err_vs_fp64"] = errs["f16"]["max_rel"]
        if not args.no_extras:
            log("bench: single-thread oracle at 1024")
            out["cpu_baseline"]["single_thread_n1024"] = oracle_single_thread(1024)

    # ------------------------------------------------------------- extras
    if not args.no_extras:
        ex = {}
        reps = 10
        dAb = torch.empty((N, N), dtype=torch.bfloat16, device=dev)
        dBb = torch.empty((N, N), dtype=torch.bfloat16, device=dev)
        mfg.round_bf16(dA32, dAb)
        mfg.round_bf16(dB32, dBb)
        dCx = dC0.clone()
        ex["bf16_n8192"] = rate_stats(flops, launch_times(
            lambda: mfg.gemm(dAb, dBb, dCx, 1.0, 1.0, mode="bf16", preconverted=True), reps))
        # context only (not this library): the vendor GEMM behind torch.matmul on the
        # same operands: FP16 (FP16 output, no C read -- less traffic than the headline)
        # and FP32 (TF32 off), beside this library's FP32 comparator
        ms = timed(lambda: torch.matmul(dA, dB), reps)
        ex["context_torch_matmul_f16_n8192"] = {"tflops": round(flops / ms / 1e9, 1),
                                                "note": "vendor library via torch.matmul, FP16 out, beta = 0"}
        torch.backends.cuda.matmul.allow_tf32 = False
        ms = timed(lambda: torch.matmul(dA32, dB32), 3, warm=1)
        ex["context_torch_matmul_f32_n8192"] = {"tflops": round(flops / ms / 1e9, 1),
                                                "note": "vendor library via torch.matmul, FP32, TF32 off"}
        ex["f32_n8192"] = rate_stats(flops, launch_times(
            lambda: mfg.gemm(dA32, dB32, dCx, 1.0, 1.0, mode="f32"), 3, warm=1))
        for mode in ("refine_a", "split3", "split4", "fp8", "bf16_split3", "bf16_split6"):
            ms = timed(lambda: mfg.gemm(dA32, dB32, dCx, 1.0, 1.0, mode=mode), 3, warm=1)
            products = {"refine_a": 2, "split3": 3, "split4": 4, "bf16_split3": 3, "bf16_split6": 6}.get(mode, 1)
            ex[f"{mode}_n8192_fp32_in"] = {"useful_tflops": round(flops / ms / 1e9, 1),
                                           "executed_tflops": round(products * flops / ms / 1e9, 1), "ms": round(ms, 3)}
        # N sweep: FP16 and BF16 (preconverted), FP32 (harmonic mean of per-launch rates)
        sweep = {"f16": {}, "bf16": {}, "f32": {}}
        for n in (1024, 2048, 4096, 16384):
            fl = 2.0 * n ** 3
            if n == 16384:  # fresh operands of the largest size
                a16 = torch.empty((n, n), dtype=torch.float16, device=dev).uniform_(-1, 1)
                b16 = torch.empty((n, n), dtype=torch.float16, device=dev).uniform_(-1, 1)
                c = torch.empty((n, n), dtype=torch.float32, device=dev).uniform_(-1, 1)
                a32, b32 = a16.float(), b16.float()
                ab, bb = a16.bfloat16(), b16.bfloat16()
            else:
                a16, b16 = dA[:n, :n].contiguous(), dB[:n, :n].contiguous()
                ab, bb = dAb[:n, :n].contiguous(), dBb[:n, :n].contiguous()
                a32, b32 = dA32[:n, :n].contiguous(), dB32[:n, :n].contiguous()
                c = dC0[:n, :n].contiguous()
            rp = 4 if n == 16384 else 20
            sweep["f16"][str(n)] = rate_stats(fl, launch_times(
                lambda: mfg.gemm(a16, b16, c, 1.0, 1.0, mode="f16", preconverted=True), rp))["tflops_hmean"]
            sweep["bf16"][str(n)] = rate_stats(fl, launch_times(
                lambda: mfg.gemm(ab, bb, c, 1.0, 1.0, mode="bf16", preconverted=True), rp))["tflops_hmean"]
            sweep["f32"][str(n)] = rate_stats(fl, launch_times(
                lambda: mfg.gemm(a32, b32, c, 1.0, 1.0, mode="f32"), 2 if n == 16384 else 5, warm=1))["tflops_hmean"]
            del a16, b16, ab, bb, a32, b32, c
        for key, row in (("f16", None), ("bf16", "bf16_n8192"), ("f32", "f32_n8192")):
            sweep[key]["8192"] = round(achieved, 2) if row is None else ex[row]["tflops_hmean"]
        ex["sweep_tflops"] = sweep
        # the one-GPU share of an eight-GPU row-panel split of N = 8192: M = 1024, N = K = 8192
        share = {}
        a_s, c_s = dA[:1024].contiguous(), dC0[:1024].contiguous()
        fl = 2.0 * 1024 * N * N
        share["f16"] = rate_stats(fl, launch_times(
            lambda: mfg.gemm(a_s, dB, c_s, 1.0, 1.0, mode="f16", preconverted=True), 20))["tflops_hmean"]
        a_s32 = dA32[:1024].contiguous()
        share["split3_fp32_in"] = rate_stats(fl, launch_times(
            lambda: mfg.gemm(a_s32, dB32, c_s, 1.0, 1.0, mode="split3"), 5, warm=1))["tflops_hmean"]
        share["f32"] = rate_stats(fl, launch_times(
            lambda: mfg.gemm(a_s32, dB32, c_s, 1.0, 1.0, mode="f32"), 5, warm=1))["tflops_hmean"]
        ex["gpu_share_m1024_n8192_k8192"] = share
        del a_s, c_s, a_s32
        # refinement study inputs (normal, sign * 2^u) at 4096 and 8192
        log("bench: precision study")
        ex["precision_fp32_in"] = precision_legs(dev, not args.no_cpu)
        log("bench: iterative-refinement solve")
        ex["solve_ir"] = solve_legs(dev)
        # refined modes from FP32: two-pass against the fused split-while-staging kernel
        log("bench: fused split")
        ex["fused_fp32_in"] = fused_legs(dev, sizes=(4096, 8192))
        # the HBM-bound steps at N x N: operand rounding, split with FP64 norms,
        # FP8 tile quantisation, FP64 error norms (algorithmic bytes per element:
        # 4 + 2, 4 + 2 + 2, 4 + 1, 4 + 8)
        h16 = torch.empty((N, N), dtype=torch.float16, device=dev)
        r16 = torch.empty((N, N), dtype=torch.float16, device=dev)
        q8 = torch.empty((N, N), dtype=torch.uint8, device=dev)
        sc = torch.empty((N // 128 + 1) * (N // 128 + 1), dtype=torch.float32, device=dev)
        nrm = torch.zeros(4, dtype=torch.float64, device=dev)
        cref = dC0.double()
        hbm = {}
        for name, fn, per_elem in (
                ("round_f16", lambda: mfg.round_f16(dA32, h16), 6),
                ("split_f16_norms", lambda: mfg.split_f16(dA32, h16, r16, nrm), 8),
                ("quantize_fp8", lambda: mfg.quantize_fp8(dA32, q8, sc), 5),
                ("error_norms", lambda: mfg.error_norms(dC0, cref, nrm), 12)):
            ms = timed(fn, 10)
            gbs = per_elem * N * N / ms / 1e6
            hbm[name] = {"us": round(ms * 1e3, 1), "gb_s": round(gbs, 1), "pct_hbm": round(100 * gbs / HBM_GBS, 1)}
        ex["hbm_steps_n8192"] = hbm
        del h16, r16, q8, sc, cref
        # batched 65536 x 16^3 and 16384 x 64^3 (FP16 in, FP32 out, alpha=1, beta=0)
        # operand sets rotate so that one pass over them (> 256 MB) outgrows the
        # L2s and the 256 MB MALL: every launch reads its operands from HBM
        def batched_leg(cnt, s, reps=20, warm=100):
            byts = cnt * (2 * 2 * s * s + 4 * s * s)
            nsets = max(1, -(-(320 << 20) // byts))
            sets = []
            for _ in range(nsets):
                a16, b16 = (torch.empty((cnt, s, s), dtype=torch.float16, device=dev).uniform_(-1, 1) for _ in range(2))
                sets.append((a16, b16, torch.empty((cnt, s, s), dtype=torch.float32, device=dev)))
            it = [0]

            def bstep():
                a16, b16, c = sets[it[0] % nsets]
                it[0] += 1
                mfg.gemm_batched(a16, b16, c, 1.0, 0.0, mode="f16")
            ms = timed(bstep, reps * nsets, warm=warm)
            del sets
            return {"gemm_per_s": round(cnt / ms * 1e3, 1), "tflops": round(2 * cnt * s ** 3 / ms / 1e9, 2),
                    "hbm_gbs": round(byts / ms / 1e6, 1), "pct_hbm": round(100 * byts / ms / 1e6 / HBM_GBS, 1),
                    "us": round(ms * 1e3, 2), "operand_sets": nsets}
        for cnt, s in ((65536, 16), (16384, 64)):
            ex[f"batched_{cnt}x{s}^3"] = batched_leg(cnt, s)
        # 16^3 batches from 2^10 to 2^18 problems (GEMM/s against the batch size)
        ex["batched_16^3_sweep_gemm_per_s"] = {str(cnt): batched_leg(cnt, 16, reps=10, warm=20)["gemm_per_s"]
                                               for cnt in (1 << 10, 1 << 12, 1 << 14, 1 << 16, 1 << 18)}
        log("bench: autotuner")
        ex["autotune_f16"] = autotune_leg(dA, dB, dev)
        log("bench: grouped tile-class tuner")
        ex["autotune_grouped"] = grouped_autotune_leg(dev)
        log("bench: grouped")
        ex.update(grouped_legs(timed, dev))
        log("bench: MFMA ceiling probe")
        ex["mfma_ceiling"] = mfma_ceiling(torch.device(dev))
        # serving: Poisson arrivals at 200 .. 5000 requests/s
        ex["serving"] = serving_legs(rates, not args.no_cpu)
        out["extras"] = ex
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
