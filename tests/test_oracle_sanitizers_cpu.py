"""The FP64 oracle's C code under the address and undefined-behaviour
sanitizers: a plain C driver runs it on seeded images (one to three block
classes, 32x32 and 64x64 windows); the result must be bitwise equal to the
oracle library the tests load."""
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLASSES = [((4, 14, 30),), ((8, 28, 12), (4, 14, 30)), ((16, 24, 8), (8, 28, 12), (4, 14, 30))]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("oracle") / "oracle_harness")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(ROOT, "tests", "oracle_harness.c"),
           os.path.join(ROOT, "oracle", "fse_oracle.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


@pytest.mark.parametrize("seed", range(6))
def test_oracle_clean_under_sanitizers(harness, tmp_path, seed):
    rng = np.random.default_rng(4000 + seed)
    W, H = int(rng.integers(8, 97)), int(rng.integers(8, 97))
    cls = CLASSES[seed % len(CLASSES)]
    img = synth.synth_image(W, H, seed=5000 + seed).astype(np.float64)
    mask = synth.mask_blocks_and_pixels(W, H, cls[-1][0], 0.2, 0.02, seed=6000 + seed)
    for (B, _, _) in cls[:-1]:  # a few fully lost squares of the larger classes
        if W >= B and H >= B:
            y, x = int(rng.integers(0, H // B)) * B, int(rng.integers(0, W // B)) * B
            mask[y:y + B, x:x + B] = 1
    (tmp_path / "img.f64").write_bytes(np.ascontiguousarray(img).tobytes())
    (tmp_path / "mask.u8").write_bytes(np.ascontiguousarray(mask).tobytes())
    args = [harness, str(tmp_path / "img.f64"), str(tmp_path / "mask.u8"), str(tmp_path / "out.f64"), str(W), str(H)]
    for c in cls:
        args += [str(v) for v in c]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:exitcode=9")
    r = subprocess.run(args, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    got = np.frombuffer((tmp_path / "out.f64").read_bytes(), np.float64).reshape(H, W)
    ref = O.image(img, mask, cls)
    assert np.array_equal(got, ref)
