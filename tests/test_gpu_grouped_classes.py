"""Tile classes of the grouped kernel (128 and 64 a side; 64 only for SPLIT4)
chosen per size bucket from the tuned table, and the grouped autotuner that
writes those entries.  Whatever class a problem runs in -- one class for
every problem, or both classes in one plan -- each result is bitwise that of
mfg_gemm on the problem alone, eagerly and on graph replays."""
import os

import numpy as np
import pytest
import torch

import paper_1803_04014_amd as mfg
import workloads
from gpu_util import DEV, dev, host, need_gpu

pytestmark = pytest.mark.gpu
MODES = ["f16", "bf16", "refine_a", "split3", "split4", "bf16_split3"]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()
    mfg.lib().mfg_tune_clear()
    yield
    mfg.lib().mfg_tune_clear()


def _bucket(x):
    return max(0, int(x).bit_length() - 1)


def _load_classes(tmp_path, mode, pick):
    """Tuned entries naming a tile class for every bucket triple up to 1023."""
    m = 32 + mfg.mode_of(mode)
    lines = [f"{m} {a} {b} {c} {pick(a, b, c)}\n" for a in range(10) for b in range(10) for c in range(10)]
    path = tmp_path / f"classes_{mode}.txt"
    path.write_text("".join(lines))
    assert mfg.lib().mfg_tune_load(str(path).encode()) == 0


def _problems(seed):
    dims = [tuple(int(x) for x in d) for d in workloads.loguniform_dims(seed, 70, 1, 400)]
    dims += [(0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 1, 1), (130, 129, 64), (64, 64, 64)]
    probs, c0 = [], []
    for i, (m, n, k) in enumerate(dims):
        A, B, C0 = workloads.normal(seed * 1000 + i, [(m, k + 3), (k, n + 5), (m, n)])
        dA, dB = dev(A), dev(B)
        if i % 5 == 0:  # rows not 16-byte aligned
            dA, dB = dA[:, 1:k + 1], dB[:, 2:n + 2]
        else:
            dA, dB = dA[:, :k], dB[:, :n]
        probs.append((dA, dB, dev(C0)))
        c0.append(C0)
    return dims, probs, c0


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("assign", ["other", "mixed"])
def test_classes_equal_solo(tmp_path, mode, assign):
    """Every problem in the other class, or classes by bucket parity."""
    classes = mfg.grouped_tile_classes(mode)
    assert classes[0] == (128 if mode in ("f16", "bf16") else 64)
    assert set(classes) <= {64, 128} and (len(classes) == 1) == (mode == "split4")
    other = classes[-1]
    pick = (lambda a, b, c: other) if assign == "other" else (lambda a, b, c: classes[(a + b) % len(classes)])
    _load_classes(tmp_path, mode, pick)
    dims, probs, c0 = _problems(61 + len(mode))
    plan = mfg.GroupedPlan(probs, mode, fp32_in=True)
    # expected classes and work items: each problem's tuned class, a class
    # with under a quarter of the flops folded into the other
    cls = [pick(_bucket(m), _bucket(n), _bucket(k)) for (m, n, k) in dims]
    fl = {t: sum(2 * m * n * k for (m, n, k), c in zip(dims, cls) if c == t) for t in classes}
    if len(classes) == 2 and all(fl.values()) and min(fl.values()) < 0.25 * sum(fl.values()):
        major = max(fl, key=fl.get)
        cls = [major] * len(cls)
    want = {}
    for (m, n, k), c in zip(dims, cls):
        if m and n:
            want[c] = want.get(c, 0) + (-(-m // c)) * (-(-n // c))
    assert plan.classes() == want
    plan.run(0.75, 0.5)
    first = [host(p[2]).copy() for p in probs]
    for i, (dA, dB, dC) in enumerate(probs):
        solo = dev(c0[i])
        mfg.gemm(dA, dB, solo, 0.75, 0.5, mode=mode)
        assert np.array_equal(first[i].view(np.uint32), host(solo).view(np.uint32)), f"{mode} {assign} {i} {dims[i]}"
    for rep in range(2):
        for (dA, dB, dC), C0 in zip(probs, c0):
            dC.copy_(dev(C0))
        plan.graph_launch(0.75, 0.5)
        torch.cuda.synchronize()
        for i in range(0, len(probs), 3):
            assert np.array_equal(host(probs[i][2]).view(np.uint32), first[i].view(np.uint32)), f"replay {rep} {i}"
    plan.close()


@pytest.mark.parametrize("mode", ["f16", "split3"])
def test_grouped_autotune_writes_the_bucket(tmp_path, mode):
    """The tuner times each class on one bucket's problems and records the
    fastest for that bucket (mode 32 + mode in the tuned table); a plan
    built afterwards runs that class."""
    M, N, K = 96, 80, 160
    probs = []
    for i in range(48):
        A, B = workloads.uniform(700 + i, [(M, K), (K, N)])
        probs.append((dev(A), dev(B), torch.zeros((M, N), dtype=torch.float32, device=DEV)))
    best, ms = mfg.grouped_autotune(probs, mode, fp32_in=True, reps=3)
    assert best in mfg.grouped_tile_classes(mode) and ms > 0
    out = tmp_path / "saved.txt"
    assert mfg.lib().mfg_tune_save(str(out).encode()) == 0
    rows = [ln.split() for ln in out.read_text().splitlines() if ln.strip() and not ln.startswith("#")]
    assert [str(32 + mfg.mode_of(mode)), str(_bucket(M)), str(_bucket(N)), str(_bucket(K)), str(best)] in rows
    # a plan built now runs that class: results still those of the problems alone
    plan = mfg.GroupedPlan(probs, mode, fp32_in=True)
    assert list(plan.classes()) == [best]
    plan.run(1.0, 0.0)
    for dA, dB, dC in probs[:6]:
        solo = torch.zeros_like(dC)
        mfg.gemm(dA, dB, solo, 1.0, 0.0, mode=mode)
        assert np.array_equal(host(dC).view(np.uint32), host(solo).view(np.uint32))
    plan.close()
