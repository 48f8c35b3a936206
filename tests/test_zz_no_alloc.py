"""fse_extrapolate_noalloc (the entry point whose device scratch is a fixed
array) against fse_extrapolate, through the C ABI: two calls in a row, the
second on a smaller image, each bitwise equal to the allocating entry point
on the same inputs and within the parity bar of the FP64 oracle; a call that
needs more scratch than the array holds is refused before anything runs; and
the calls take no device memory (free device memory unchanged)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

pytestmark = pytest.mark.gpu


def _inputs(W, H, seed):
    img = synth.synth_image(W, H, seed=seed, period_max=128.0)
    mask = synth.mask_blocks_and_pixels(W, H, 4, 0.25, 0.01, seed=seed + 1)
    return img, mask


def _both(img, mask, **kw):
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(img).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    p = fse.fse_params_default(**kw)
    ref = torch.full_like(ti, -1.0)
    fse.fse_extrapolate(ti, tm, p, ref)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = torch.full_like(ti, -2.0)
    fse.fse_extrapolate_noalloc(ti, tm, p, got)
    torch.cuda.synchronize()
    st = fse.fse_last_stats()
    free1 = torch.cuda.mem_get_info()[0]
    return ref.cpu().numpy(), got.cpu().numpy(), st, free0, free1


def _setup_call():
    # the first call on a device sets up its copy of the scratch array (the
    # runtime loads the array with its code object then); later calls
    # allocate nothing
    img, mask = _inputs(32, 32, 499)
    _both(img, mask)


def test_noalloc_equals_allocating_entry_point_twice_second_smaller():
    classes = ((4, 14, 100),)
    _setup_call()
    for (W, H, seed) in ((384, 256, 501), (200, 136, 503)):
        img, mask = _inputs(W, H, seed)
        print(f"case {W}x{H} seed {seed}", flush=True)
        ref, got, st, free0, free1 = _both(img, mask)
        assert st["device_error"] == 0, st
        assert np.array_equal(got, ref), f"{W}x{H}: no-alloc result differs from fse_extrapolate"
        assert free1 == free0, (free0, free1)
        m = mask.astype(bool)
        orc = O.image(img, mask, classes)
        assert np.array_equal(got[~m], img[~m])
        assert np.abs(got.astype(np.float64) - orc)[m].max() <= 1e-3


def test_noalloc_tiled_and_64_window_classes():
    # the tile framework and a launch with 64 x 64 windows (eight-wave
    # workgroups) through the same scratch
    W, H = 160, 120
    img = synth.synth_image(W, H, seed=511, period_max=64.0)
    mask = synth.mask_blocks(W, H, 8, 0.08, seed=512) | synth.mask_blocks_and_pixels(W, H, 4, 0.05, 0.005, seed=513)
    cls = ((8, 28, 30), (4, 14, 40))
    for kw in (dict(classes=cls), dict(classes=((4, 14, 60),), tiling=1, n_tiles=6, overlap=16, align=16)):
        ref, got, st, _, _ = _both(img, mask, **kw)
        assert st["device_error"] == 0
        assert np.array_equal(got, ref)


def test_noalloc_refuses_what_does_not_fit():
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    # 8 bytes per pixel of FP64 working copy alone exceed the 32 MiB array
    W, H = 2100, 2100
    ti = torch.zeros((H, W), dtype=torch.float32, device=dev)
    tm = torch.zeros((H, W), dtype=torch.uint8, device=dev)
    tm[::64, ::64] = 1
    out = torch.full_like(ti, 7.0)
    with pytest.raises(fse.FseError) as ei:
        fse.fse_extrapolate_noalloc(ti, tm, fse.fse_params_default(), out)
    assert ei.value.status == fse.FSE_ERR_BUDGET
    torch.cuda.synchronize()
    assert bool((out == 7.0).all()), "a refused call wrote its output"
    # tiles whose extended regions together exceed the array: refused after
    # planning, before anything is enqueued
    W, H = 1400, 1400  # 1.96 Mpixel: 15.7 MB whole; 64 tiles with d = 96 grow it past 32 MiB
    ti = torch.zeros((H, W), dtype=torch.float32, device=dev)
    tm = torch.zeros((H, W), dtype=torch.uint8, device=dev)
    tm[::40, ::40] = 1
    out = torch.full_like(ti, 7.0)
    p = fse.fse_params_default(tiling=1, n_tiles=64, overlap=96, align=16)
    with pytest.raises(fse.FseError) as ei:
        fse.fse_extrapolate_noalloc(ti, tm, p, out)
    assert ei.value.status == fse.FSE_ERR_BUDGET
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
