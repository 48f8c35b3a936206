"""Seeded random cases against the oracle: image sizes from 1 to 160 pixels,
masks mixing lost blocks, isolated pixels and row defects, one to three
block classes (32x32 and 64x64 windows), whole-image and both tiled modes,
every schedule and every block width."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

pytestmark = pytest.mark.gpu

TIGHT = 1e-3
CLASSES = [((4, 14, 40),), ((8, 28, 24), (4, 14, 40)), ((16, 24, 16), (8, 28, 24), (4, 14, 40))]


def case(seed):
    rng = np.random.default_rng(1000 + seed)
    W = int(rng.integers(1, 161))
    H = int(rng.integers(1, 161))
    cls = CLASSES[int(rng.integers(len(CLASSES)))]
    img = synth.synth_image(W, H, seed=2000 + seed, period_max=float(rng.choice([16.0, 64.0, 256.0])))
    mask = np.zeros((H, W), np.uint8)
    for (B, _, _) in cls:  # aligned squares of each class's size
        nb = (H // B) * (W // B)
        if nb:
            k = int(rng.integers(0, max(1, nb // 4) + 1))
            for q in rng.choice(nb, size=min(k, nb), replace=False):
                y, x = divmod(int(q), W // B)
                mask[y * B:(y + 1) * B, x * B:(x + 1) * B] = 1
    mask[rng.random((H, W)) < rng.uniform(0, 0.03)] = 1  # isolated pixels
    for _ in range(int(rng.integers(0, 3))):  # row defects
        mask[int(rng.integers(H)), :] = 1
    mode = int(rng.integers(3))  # 0 whole, 1 compact tiles, 2 vertical stripes
    Bmax = cls[0][0]
    N = int(rng.integers(1, 9))
    d = int(rng.integers(0, 40))
    align = Bmax * int(rng.integers(1, 3))
    schedule = int(rng.choice(3, p=[0.6, 0.2, 0.2]))  # persistent, wavefront, one launch per block
    waves = int(rng.choice([0, 1, 2, 4]))
    return img, mask, cls, mode, N, d, align, schedule, waves


@pytest.mark.parametrize("seed", range(48))
def test_random_case_matches_oracle(seed):
    import torch
    from paper_2207_00238_amd import fse
    img, mask, cls, mode, N, d, align, schedule, waves = case(seed)
    H, W = mask.shape
    print(f"seed {seed}: {W}x{H}, classes {[c[0] for c in cls]}, mode {mode}, N {N}, d {d}, align {align}, "
          f"schedule {schedule}, waves {waves}, lost {int(mask.sum())}", flush=True)
    kw = dict(classes=cls, schedule=schedule, block_waves=waves)
    if mode == 0:
        ref = O.image(img, mask, cls)
        p = fse.fse_params_default(**kw)
    else:
        N = min(N, W * H)
        ref = O.image_tiled(img, mask, cls, N, d, align, vertical=(mode == 2))
        p = fse.fse_params_default(**kw, tiling=fse.FSE_TILED if mode == 1 else fse.FSE_TILED_VERTICAL,
                                   n_tiles=N, overlap=d, align=align)
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    out = torch.full_like(ti, -12345.0)
    fse.fse_extrapolate(ti, tm, p, out)
    torch.cuda.synchronize()
    st = fse.fse_last_stats()
    assert st["device_error"] == 0
    got = out.cpu().numpy()
    m = mask.astype(bool)
    assert np.array_equal(got[~m], img[~m])
    if m.any():
        assert np.abs(got.astype(np.float64) - ref)[m].max() <= TIGHT
