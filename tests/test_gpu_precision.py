"""Reduced-precision modes (FP32 and BF16x3 DFT with an FP32 selection loop)
held to the stated bar against the FP64 oracle:

  * max |dpixel| <= 0.5 grey levels on >= 99.9 % of the lost pixels;
  * |dPSNR| <= 0.01 dB;
  * a basis selection may leave the oracle's sequence only where the
    oracle's energies of the two choices differ by < 1e-5 relative (exact
    mirror ties, which give the same real output, are followed).

The FP64 path is the parity path (tests/test_gpu_parity.py); these tests
record where each reduced mode meets the bar and where it does not.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

from parity import compare_traces, pixel_report

pytestmark = pytest.mark.gpu


def _run(img, mask, classes, precision, trace=False, **kw):
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).to(dev)
    tm = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(dev)
    out = torch.full_like(ti, -12345.0)
    p = fse.fse_params_default(classes=classes, precision=precision, **kw)
    sel = None
    if trace:
        nb = len(O.plan(mask, classes)[0])
        K = max(c[2] for c in classes)
        sel = torch.full((max(nb, 1), K), -1, dtype=torch.int32, device=dev)
        p.trace_sel = sel.data_ptr()
        p.trace_stride = K
        p.trace_capacity = nb
    fse.fse_extrapolate(ti, tm, p, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (sel.cpu().numpy() if trace else None)


def _at_the_bar(img, mask, classes, precision):
    ref, tr = O.image(img, mask, classes, trace=True)
    got, sel = _run(img, mask, classes, precision, trace=True)
    m = mask.astype(bool)
    assert np.array_equal(got[~m], np.asarray(img, np.float32)[~m])
    rep = pixel_report(got, ref, img, mask)
    B, b, K = classes[-1]
    cmp = compare_traces(sel, tr, B + 2 * b, K, tol=1e-5)
    print("precision", precision, rep, {k: v for k, v in cmp.items() if k != "bad_examples"}, flush=True)
    return rep, cmp


@pytest.mark.parametrize("precision", [1, 2])
def test_reduced_precision_exact_patterns(precision):
    H, W = 64, 96
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    img = (100 + 30.0 * (-1.0) ** (x + y)).astype(np.float32)
    mask = synth.mask_blocks(W, H, 4, 0.3, seed=5)
    got, _ = _run(img, mask, ((4, 14, 20),), precision, gamma=1.0)
    m = mask.astype(bool)
    # two basis functions: recovered up to the arithmetic's rounding
    tol = 2e-3 if precision == 1 else 0.05
    assert np.abs(got - img)[m].max() < tol


# FP32 meets the bar on the 128 x 128 workload.  BF16x3 does not: its hi/lo
# split drops the lo*lo product, a relative error of ~2^-16 per product
# (FP32: 2^-24), and the greedy selection cascades along the raster chain
# (measured on MI355X: 92.1 % of lost pixels within 0.5, max 3.03, 47 blocks
# leave the oracle's sequence at gaps >= 1e-5).  Its case is a strict xfail:
# the bar stays the stated one, and a change that makes BF16x3 meet it shows.
@pytest.mark.parametrize("precision", [
    1,
    pytest.param(2, marks=pytest.mark.xfail(strict=True, reason="BF16x3 misses the stated bar on this workload")),
])
def test_reduced_precision_small_workload_at_the_stated_bar(precision):
    # the 128 x 128 workload (205 lost 4 x 4 blocks, K = 100)
    wl = synth.workload("small")
    rep, cmp = _at_the_bar(wl.image, wl.mask, wl.classes, precision)
    assert rep["frac_le_half"] >= 0.999, rep
    assert rep["dpsnr"] <= 0.01, rep
    assert cmp["divergences_bad"] == 0, cmp
