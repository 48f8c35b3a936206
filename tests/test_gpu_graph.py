"""Prepared plans replayed as HIP graphs: every replay equals the eager
result, with eager work and synchronisations between replays, for changing
image contents under fixed masks."""
import numpy as np
import pytest

from oracle import oracle as O

from paper_2207_00238_amd import synth

pytestmark = pytest.mark.gpu


def test_plan_replays_match_eager():
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    sizes = [(120, 96), (64, 150)]
    masks = [torch.from_numpy(synth.mask_blocks_and_pixels(W, H, 4, 0.25, 0.01, seed=70 + i)).to(dev)
             for i, (W, H) in enumerate(sizes)]
    p = fse.fse_params_default(classes=((4, 14, 40),))
    plan = fse.fse_plan_create(masks, p)
    try:
        for rep in range(4):
            imgs = [torch.from_numpy(synth.synth_image(W, H, seed=200 + 10 * rep + i)).to(dev)
                    for i, (W, H) in enumerate(sizes)]
            eager = [torch.empty_like(t) for t in imgs]
            fse.fse_extrapolate_batch(imgs, masks, p, eager)
            torch.cuda.synchronize()
            outs = [torch.full_like(t, -7.0) for t in imgs]
            fse.fse_plan_execute(plan, imgs, outs)
            torch.cuda.synchronize()
            for e, o in zip(eager, outs):
                assert torch.equal(e, o), f"replay {rep} differs from the eager result"
            # unrelated eager work between replays
            scratch = torch.randn(1 << 16, device=dev).sum().item()
            assert np.isfinite(scratch)
    finally:
        fse.fse_plan_destroy(plan)


def test_plan_rejects_mismatched_images():
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    m = torch.from_numpy(synth.mask_blocks(64, 64, 4, 0.2, seed=5)).to(dev)
    plan = fse.fse_plan_create([m], fse.fse_params_default(classes=((4, 14, 10),)))
    try:
        img = torch.zeros((64, 32), dtype=torch.float32, device=dev)
        with pytest.raises(fse.FseError):
            fse.fse_plan_execute(plan, [img], [torch.empty_like(img)])
    finally:
        fse.fse_plan_destroy(plan)


def test_autotune_returns_equivalent_schedule():
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    wl = synth.workload("small")
    img = torch.from_numpy(wl.image).to(dev)
    msk = torch.from_numpy(wl.mask).to(dev)
    p = fse.fse_params_default(classes=wl.classes, block_waves=0)
    out_a = torch.empty_like(img)
    best = fse.fse_autotune([img], [msk], p, [out_a])
    assert best.block_waves in (1, 2, 4) and best.workgroups >= 0
    out_b = torch.empty_like(img)
    fse.fse_extrapolate(img, msk, best, out_b)
    torch.cuda.synchronize()
    assert torch.equal(out_a, out_b)
    # cached: the second call returns the same schedule
    best2 = fse.fse_autotune([img], [msk], p, [out_a])
    assert (best2.block_waves, best2.workgroups) == (best.block_waves, best.workgroups)


def test_plan_stats_reports_the_error_word(monkeypatch):
    # fse_plan_stats waits for the last execution and reports its error word:
    # set when the plan was prepared with a (host-forced, zero) wait limit,
    # clear for a plan prepared with the normal limit
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    W, H = 256, 192
    img = torch.from_numpy(synth.synth_image(W, H, seed=91, period_max=128.0)).to(dev)
    msk = torch.from_numpy(synth.mask_blocks_and_pixels(W, H, 4, 0.25, 0.01, seed=92)).to(dev)
    p = fse.fse_params_default(classes=((4, 14, 30),), workgroups=256)
    out = torch.empty_like(img)
    for limit, expect_error in (("0", True), (None, False)):
        if limit is None:
            monkeypatch.delenv("FSE_WAIT_LIMIT_US", raising=False)
        else:
            monkeypatch.setenv("FSE_WAIT_LIMIT_US", limit)
        plan = fse.fse_plan_create([msk], p)
        try:
            assert fse.fse_plan_stats(plan)["device_error"] == 0  # before any execution
            fse.fse_plan_execute(plan, [img], [out])
            st = fse.fse_plan_stats(plan)
            assert st["n_blocks"] > 0
            assert (st["device_error"] != 0) == expect_error
        finally:
            fse.fse_plan_destroy(plan)


def test_autotuned_tile_count_matches_the_tile_oracle():
    # n_tiles = 0 asks the tuner for the tile count N of Algorithm 1 as well;
    # the tuned schedule's result is the tile framework's with that N
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    W, H = 200, 136
    imgn = synth.synth_image(W, H, seed=951, period_max=128.0)
    mskn = synth.mask_blocks_and_pixels(W, H, 4, 0.25, 0.01, seed=952)
    img = torch.from_numpy(imgn).to(dev)
    msk = torch.from_numpy(mskn).to(dev)
    cls = ((4, 14, 40),)
    p = fse.fse_params_default(classes=cls, tiling=fse.FSE_TILED, n_tiles=0, overlap=16, align=16)
    out = torch.empty_like(img)
    best = fse.fse_autotune([img], [msk], p, [out])
    assert best.n_tiles in (16, 32, 64, 128, 256), best.n_tiles
    assert best.overlap == 16
    got = torch.full_like(img, -1.0)
    fse.fse_extrapolate(img, msk, best, got)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref = O.image_tiled(imgn, mskn, cls, best.n_tiles, 16, 16)
    m = mskn.astype(bool)
    assert np.array_equal(got[~m], imgn[~m])
    assert np.abs(got - ref)[m].max() <= 1e-3
    # a plain call with n_tiles = 0 is refused (only the tuner picks N)
    with pytest.raises(fse.FseError):
        fse.fse_extrapolate(img, msk, p, torch.empty_like(img))


def test_autotune_overlapped_keeps_results():
    # the schedule for consecutive calls in flight on three streams: the same
    # output as the default schedule, bit for bit
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    imgs, msks = [], []
    for i in range(3):
        imgs.append(torch.from_numpy(synth.synth_image(160, 120, seed=961 + 2 * i, period_max=128.0)).to(dev))
        msks.append(torch.from_numpy(synth.mask_blocks_and_pixels(160, 120, 4, 0.25, 0.01, seed=962 + 2 * i)).to(dev))
    p = fse.fse_params_default(classes=((4, 14, 40),))
    outs = [torch.empty_like(t) for t in imgs]
    best = fse.fse_autotune_overlapped(imgs, msks, p, outs, 3)
    torch.cuda.synchronize()
    ref = [torch.empty_like(t) for t in imgs]
    fse.fse_extrapolate_batch(imgs, msks, p, ref)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(outs, ref))
    got = [torch.empty_like(t) for t in imgs]
    fse.fse_extrapolate_batch(imgs, msks, best, got)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(got, ref))


def test_autotune_cache_keys_on_the_mask_structure():
    # same sizes and parameters, masks of another structure (another number
    # of blocks): tuned anew, so the second mask's call takes as long as a
    # tuning run, while repeating the first mask returns from the cache
    import time
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    W, H = 192, 160
    img = torch.from_numpy(synth.synth_image(W, H, seed=971, period_max=128.0)).to(dev)
    m1 = torch.from_numpy(synth.mask_blocks(W, H, 4, 0.2, seed=972)).to(dev)
    m2 = torch.from_numpy(synth.mask_blocks(W, H, 4, 0.05, seed=973)).to(dev)
    p = fse.fse_params_default(classes=((4, 14, 20),), gamma=0.55)
    out = torch.empty_like(img)

    def timed(m):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fse.fse_autotune([img], [m], p, [out])
        return time.perf_counter() - t0

    first = timed(m1)
    again = timed(m1)
    other = timed(m2)
    assert again < 0.5 * first, (first, again)
    assert other > 2 * again, (again, other)
