"""The library's host planner (fse_plan.cpp) on the CPU, built with the
address and undefined-behaviour sanitizers: on seeded masks it finds the same
processing blocks and owners as the oracle, and its dependency levels order
every dependency of the oracle's raster semantics (so tickets sorted by level
never wait on a later ticket)."""
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_00238_amd", "csrc")
CLASSES = [((4, 14, 1),), ((8, 28, 1), (4, 14, 1)), ((16, 24, 1), (8, 28, 1), (4, 14, 1))]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("plan") / "plan_harness")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I" + CSRC, os.path.join(ROOT, "tests", "plan_harness.cpp"),
           os.path.join(CSRC, "fse_plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


def _mask(seed):
    rng = np.random.default_rng(3000 + seed)
    W, H = int(rng.integers(1, 121)), int(rng.integers(1, 121))
    cls = CLASSES[int(rng.integers(len(CLASSES)))]
    mask = np.zeros((H, W), np.uint8)
    for (B, _, _) in cls:
        nb = (H // B) * (W // B)
        if nb:
            for q in rng.choice(nb, size=min(int(rng.integers(0, nb // 3 + 1)), nb), replace=False):
                y, x = divmod(int(q), W // B)
                mask[y * B:(y + 1) * B, x * B:(x + 1) * B] = 1
    mask[rng.random((H, W)) < rng.uniform(0, 0.04)] = 1
    if H > 2 and rng.random() < 0.5:
        mask[int(rng.integers(H)), :] = 1
    return mask, cls


def _run(exe, tmp_path, mask, cls, opt=None):
    H, W = mask.shape
    f = tmp_path / "mask.u8"
    f.write_bytes(np.ascontiguousarray(mask).tobytes())
    args = [exe, str(f), str(W), str(H)]
    if opt is not None:
        args += ["opt", repr(float(opt[0])), repr(float(opt[1]))]
    for (B, b, _) in cls:
        args += [str(B), str(b)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=9")
    r = subprocess.run(args, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = r.stdout.split("\n")
    n = int(lines[0].split()[1])
    blocks = np.array([[int(v) for v in l.split()] for l in lines[1:1 + n]], np.int64).reshape(n, 4)
    fw, fh = (int(v) for v in lines[1 + n].split()[1:3])
    owner = np.array([[int(v) for v in l.split()] for l in lines[2 + n:2 + n + fh]], np.int64).reshape(fh, fw)
    return blocks, owner


@pytest.mark.parametrize("seed", range(16))
def test_planner_matches_oracle(harness, tmp_path, seed):
    mask, cls = _mask(seed)
    blocks, cell_owner = _run(harness, tmp_path, mask, cls)
    y, x, c, owner = O.plan(mask, cls)
    assert len(blocks) == len(y)
    assert np.array_equal(blocks[:, 0], y) and np.array_equal(blocks[:, 1], x) and np.array_equal(blocks[:, 2], c)
    Bmin = cls[-1][0]
    ly, lx = np.nonzero(mask)
    assert np.array_equal(cell_owner[ly // Bmin, lx // Bmin], owner[ly, lx])
    level = blocks[:, 3]
    for j, preds in enumerate(O.dependencies(mask, cls)):
        for i in preds:
            assert level[i] < level[j], (i, j)


def test_planner_on_the_1080p_mask(harness, tmp_path):
    # the benchmark's mask: same blocks as the oracle, and the levels' depth is
    # the oracle's dependency depth
    wl = synth.workload("hd", 0)
    blocks, _ = _run(harness, tmp_path, wl.mask, wl.classes)
    y, x, c, _ = O.plan(wl.mask, wl.classes)
    assert np.array_equal(blocks[:, 0], y) and np.array_equal(blocks[:, 1], x)
    assert blocks[:, 3].max() + 1 == 1259


# ---------------------------------------------------------------------------
# the optimised processing order (Sec. II): the planner's order is the
# oracle's, and its levels order every dependency of that order
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
def test_planner_priority_order_matches_oracle(harness, tmp_path, seed):
    mask, cls = _mask(seed)
    rho, delta = ((0.8, 0.5), (1.0, 0.5), (0.9, 0.7))[seed % 3]
    if mask.shape[0] > 20 and mask.shape[1] > 20:
        mask[5:5 + mask.shape[0] // 3, 3:3 + mask.shape[1] // 2] = 1  # a larger hole
    blocks, cell_owner = _run(harness, tmp_path, mask, cls, opt=(rho, delta))
    y, x, c, owner = O.plan(mask, cls)
    order = O.priority_order(mask, cls, rho=rho, delta=delta)
    assert len(blocks) == len(order)
    assert np.array_equal(blocks[:, 0], y[order]) and np.array_equal(blocks[:, 1], x[order])
    assert np.array_equal(blocks[:, 2], c[order])
    rank = np.argsort(order)
    Bmin = cls[-1][0]
    ly, lx = np.nonzero(mask)
    assert np.array_equal(cell_owner[ly // Bmin, lx // Bmin], rank[owner[ly, lx]])
    level = blocks[:, 3]  # by processing rank
    preds = O.dependencies(mask, cls, order=order)
    for j, pj in enumerate(preds):
        for i in pj:
            assert level[rank[i]] < level[rank[j]], (i, j)
    # and exactly the longest chain of the kernel's waits: two blocks wait on
    # each other when the bounding box of either one's lost pixels meets the
    # other's window (brute force over all pairs, in processing order)
    n = len(order)
    box = np.zeros((n, 4), np.int64)
    for b in range(n):
        ys, xs = np.nonzero(owner == b)
        box[b] = (ys.min(), xs.min(), ys.max() + 1, xs.max() + 1)
    win = np.array([(y[b] - cls[c[b]][1], x[b] - cls[c[b]][1], y[b] + cls[c[b]][0] + cls[c[b]][1],
                     x[b] + cls[c[b]][0] + cls[c[b]][1]) for b in range(n)], np.int64).reshape(n, 4)

    def meet(a, b):
        return (a[:, 0] < b[:, 2]) & (b[:, 0] < a[:, 2]) & (a[:, 1] < b[:, 3]) & (b[:, 1] < a[:, 3])

    want = np.zeros(n, np.int64)
    for k in range(n):
        j = order[k]
        earlier = order[:k]
        if k:
            hit = meet(box[earlier], win[[j] * k]) | meet(box[[j] * k], win[earlier])
            if hit.any():
                want[j] = want[earlier[hit]].max() + 1
    assert np.array_equal(level, want[order])


def test_planner_priority_order_on_the_1080p_mask(harness, tmp_path):
    # the benchmark's mask: the same order as the oracle at full size
    wl = synth.workload("hd", 0)
    blocks, _ = _run(harness, tmp_path, wl.mask, wl.classes, opt=(0.8, 0.5))
    y, x, _, _ = O.plan(wl.mask, wl.classes)
    order = O.priority_order(wl.mask, wl.classes)
    assert np.array_equal(blocks[:, 0], y[order]) and np.array_equal(blocks[:, 1], x[order])
    print("levels: optimised order", blocks[:, 3].max() + 1)
