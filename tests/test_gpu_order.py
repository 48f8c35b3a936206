"""GPU parity of the optimised processing order (Sec. II; FSE_ORDER_OPTIMIZED)
against the FP64 oracle processing the blocks in its own optimised order:
whole images under every schedule, mixed block classes with 64 x 64
windows, the tile framework (each tile in its own order), and the selection
traces, which the library indexes by processing rank."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

from parity import compare_traces, pixel_report

pytestmark = pytest.mark.gpu

TIGHT = 1e-3


def _holes_mask(W, H, seed):
    # random blocks and pixels plus large holes, where the order matters most
    rng = np.random.default_rng(seed)
    mask = synth.mask_blocks_and_pixels(W, H, 4, 0.2, 0.01, seed=seed)
    for _ in range(3):
        h, w = int(rng.integers(12, 33)), int(rng.integers(12, 41))
        y, x = int(rng.integers(0, H - h)), int(rng.integers(0, W - w))
        mask[y:y + h, x:x + w] = 1
    return mask


def _run(img, mask, classes, trace=False, **kw):
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).to(dev)
    tm = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(dev)
    out = torch.full_like(ti, -12345.0)
    p = fse.fse_params_default(classes=classes, order=fse.FSE_ORDER_OPTIMIZED, **kw)
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
    return out.cpu().numpy(), (sel.cpu().numpy() if trace else None), fse.fse_last_stats()


def _check(img, mask, classes, **kw):
    order = O.priority_order(mask, classes)
    ref, tr = O.image(img, mask, classes, order=order, trace=True)
    got, sel, st = _run(img, mask, classes, trace=True, **kw)
    print("case", img.shape, classes, kw, st, flush=True)
    assert st["device_error"] == 0
    m = mask.astype(bool)
    assert np.array_equal(got[~m], np.asarray(img, np.float32)[~m])
    rep = pixel_report(got, ref, img, mask)
    # GPU trace rows are processing ranks; the oracle's are raster indices
    rank = np.argsort(order)
    cb = O.plan(mask, classes)[2]
    M = np.array([classes[c][0] + 2 * classes[c][1] for c in cb], dtype=np.int64)
    Ks = np.array([classes[c][2] for c in cb], dtype=np.int64)
    cmp = compare_traces(sel[rank], tr, M, Ks)
    print(rep, cmp, flush=True)
    assert cmp["divergences_bad"] == 0, cmp
    assert rep["max_abs"] <= TIGHT, rep
    return got, ref, st


@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_optimized_order_all_schedules(schedule):
    W, H = 144, 104
    img = synth.synth_image(W, H, seed=801, period_max=128.0)
    mask = _holes_mask(W, H, 802)
    _, _, st = _check(img, mask, ((4, 14, 60),), schedule=schedule)
    if schedule == 0:
        # the levels of the optimised order's DAG: far fewer than the blocks
        assert st["wavefront_keys"] < st["n_blocks"] // 3


def test_optimized_order_small_workload():
    wl = synth.workload("small")
    _check(wl.image, wl.mask, wl.classes)


@pytest.mark.parametrize("waves", [1, 2])
def test_optimized_order_block_waves(waves):
    W, H = 120, 96
    img = synth.synth_image(W, H, seed=811, period_max=64.0)
    mask = _holes_mask(W, H, 812)
    _check(img, mask, ((4, 14, 50),), block_waves=waves)


def test_optimized_order_mixed_classes_64_windows():
    W, H = 160, 128
    img = synth.synth_image(W, H, seed=821, period_max=64.0)
    mask = synth.mask_mixed(W, H, seed=822, frac8=0.1, frac16=0.05, row_fraction=0.02)
    mask[40:72, 60:100] = 1
    _check(img, mask, ((16, 24, 40), (8, 28, 40), (4, 14, 30)))


def test_optimized_order_tiled():
    W, H = 200, 136
    img = synth.synth_image(W, H, seed=831, period_max=128.0)
    mask = _holes_mask(W, H, 832)
    cls = ((4, 14, 40),)
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(img).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    out = torch.full_like(ti, -12345.0)
    p = fse.fse_params_default(classes=cls, tiling=fse.FSE_TILED, n_tiles=6, overlap=16, align=16,
                               order=fse.FSE_ORDER_OPTIMIZED)
    fse.fse_extrapolate(ti, tm, p, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = O.image_tiled(img, mask, cls, 6, 16, 16, optimized_order=True)
    m = mask.astype(bool)
    assert np.array_equal(got[~m], img[~m])
    assert np.abs(got - ref)[m].max() <= TIGHT


def test_optimized_order_batch_and_ragged():
    # two images of different sizes in one launch, one of them ragged
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    cls = ((4, 14, 40),)
    cases = [(150, 93, 841), (96, 64, 843)]
    imgs, masks, outs, refs = [], [], [], []
    for (W, H, seed) in cases:
        img = synth.synth_image(W, H, seed=seed, period_max=128.0)
        mask = _holes_mask(W, H, seed + 1)
        imgs.append(torch.from_numpy(img).to(dev))
        masks.append(torch.from_numpy(mask).to(dev))
        outs.append(torch.full_like(imgs[-1], -1.0))
        refs.append((O.image(img, mask, cls, order=O.priority_order(mask, cls)), img, mask))
    p = fse.fse_params_default(classes=cls, order=fse.FSE_ORDER_OPTIMIZED)
    fse.fse_extrapolate_batch(imgs, masks, p, outs)
    torch.cuda.synchronize()
    for o, (ref, img, mask) in zip(outs, refs):
        got = o.cpu().numpy()
        m = mask.astype(bool)
        assert np.array_equal(got[~m], img[~m])
        assert np.abs(got - ref)[m].max() <= TIGHT
