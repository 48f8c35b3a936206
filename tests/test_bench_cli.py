"""The benchmark's command line on the CPU: one GPU only, argument checks
before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_streams_must_be_positive():
    r = _run("--streams", "0")
    assert r.returncode != 0
    assert "--streams" in r.stderr


def test_ssim_closed_forms():
    # identical images: 1; constant images a and b: (2ab + C1) / (a^2 + b^2 + C1)
    # (the variance terms are 0 and the structure factor C2 / C2 = 1)
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 255, (64, 80))
    assert abs(bench.ssim(x, x) - 1.0) < 1e-12
    a, b = 100.0, 140.0
    c1 = (0.01 * 255) ** 2
    want = (2 * a * b + c1) / (a * a + b * b + c1)
    assert abs(bench.ssim(np.full((40, 40), a), np.full((40, 40), b)) - want) < 1e-12
    # more noise, lower similarity
    n = rng.normal(0, 1, x.shape)
    s10, s40 = bench.ssim(x + 10 * n, x), bench.ssim(x + 40 * n, x)
    assert s40 < s10 < 1.0
