"""Reduced-precision modes (FP32 and BF16x3 DFT with an FP32 selection loop).

They are measured against the FP64 oracle, not held to the FP64 path's bar:
the greedy selection turns small spectral errors into different basis
choices, which then propagate through the reconstructed support of later
blocks.  The tests check that each mode computes the method (single-basis
images are exact, random images stay close in PSNR) and record its error.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

from parity import pixel_report

pytestmark = pytest.mark.gpu


def _run(img, mask, classes, precision, **kw):
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).to(dev)
    tm = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(dev)
    out = torch.full_like(ti, -12345.0)
    p = fse.fse_params_default(classes=classes, precision=precision, **kw)
    fse.fse_extrapolate(ti, tm, p, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", [1, 2])
def test_reduced_precision_exact_patterns(precision):
    H, W = 64, 96
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    img = (100 + 30.0 * (-1.0) ** (x + y)).astype(np.float32)
    mask = synth.mask_blocks(W, H, 4, 0.3, seed=5)
    got = _run(img, mask, ((4, 14, 20),), precision, gamma=1.0)
    m = mask.astype(bool)
    # two basis functions: recovered up to the arithmetic's rounding
    tol = 2e-3 if precision == 1 else 0.05
    assert np.abs(got - img)[m].max() < tol


@pytest.mark.parametrize("precision", [1, 2])
def test_reduced_precision_small_workload(precision):
    wl = synth.workload("small")
    ref = O.image(wl.image, wl.mask, wl.classes)
    got = _run(wl.image, wl.mask, wl.classes, precision)
    m = wl.mask.astype(bool)
    assert np.array_equal(got[~m], wl.image[~m])
    rep = pixel_report(got, ref, wl.image, wl.mask)
    print("precision", precision, rep)
    assert np.isfinite(got).all()
    # PSNR against the ground truth within a few tenths of a dB of the FP64 result
    assert rep["dpsnr"] < 0.5
