"""The optimised processing order of the oracle (Sec. II: large lost areas
are closed from their margins towards their centre; the rule is reading R17:
each step takes the remaining block whose support window offers the largest
share of usable weight, ties to the raster-earlier block), pinned by

  * a square hole with rho = 1, where the shares are pixel counts and the
    first steps follow by hand, and the hole closes from the margin inwards;
  * a brute-force check of the rule at every step (shares summed again over
    whole windows with NumPy from the status map);
  * the processing semantics: any order that respects the dependencies of
    the optimised order gives the bitwise identical image;
  * mistakes planted in a copy of the oracle, each rejected by a pin above.
"""
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

ORACLE_C = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "fse_oracle.c")

# a 40 x 40 hole (10 x 10 blocks of 4 x 4) inside a 128 x 128 image
HOLE0 = 44


def _hole():
    mask = np.zeros((128, 128), np.uint8)
    mask[HOLE0:HOLE0 + 40, HOLE0:HOLE0 + 40] = 1
    return mask


def _cells(mask, cls, order):
    y, x, _, _ = O.plan(mask, cls)
    return [(int(y[i] - HOLE0) // 4, int(x[i] - HOLE0) // 4) for i in order]


def _hand_pin():
    # rho = 1, delta = 0.5: a window's share is (known + recon / 2) / 1024.
    # Block (i, j) of the hole sees the hole's rows 4i-14 .. 4i+17 (clipped
    # to 0..39), so the lost pixels in its window are 18 x 18 = 324 for a
    # corner, 18 x 22 = 396 for the neighbours of a corner, more inside:
    #   steps 1-4: the four corners (700 known each), raster order;
    #   step 5: (0,1) -- 628 known + 8 from the 16 pixels of (0,0), tied with
    #     the seven other neighbours of a corner, raster-first;
    #   step 6: (1,0) -- 628 + 8 + 8: it also sees the pixels of (0,1),
    #     while (0,8) has 628 + 8.
    mask = _hole()
    cls = ((4, 14, 1),)
    cells = _cells(mask, cls, O.priority_order(mask, cls, rho=1.0, delta=0.5))
    return cells


def test_square_hole_by_hand():
    cells = _hand_pin()
    assert cells[:6] == [(0, 0), (0, 9), (9, 0), (9, 9), (0, 1), (1, 0)], cells[:6]


@pytest.mark.parametrize("rho", [1.0, 0.8])
def test_square_hole_closes_from_the_margin(rho):
    mask = _hole()
    cls = ((4, 14, 1),)
    cells = _cells(mask, cls, O.priority_order(mask, cls, rho=rho))
    ring = np.array([min(i, j, 9 - i, 9 - j) for (i, j) in cells])
    assert sorted(cells) == [(i, j) for i in range(10) for j in range(10)]
    # the outer ring first, the centre last
    assert (ring[:16] == 0).all()
    assert set(cells[-4:]) == {(4, 4), (4, 5), (5, 4), (5, 5)}
    # and the rings by and large in turn: the mean ring of each quarter grows
    q = [ring[k * 25:(k + 1) * 25].mean() for k in range(4)]
    assert q[0] < q[1] < q[2] < q[3], q


def _weights(M, rho, delta):
    c = (M - 1) / 2
    m = np.arange(M)[:, None] - c
    n = np.arange(M)[None, :] - c
    wk = rho ** np.sqrt(m * m + n * n)
    return wk, delta * wk


def _check_rule(mask, cls, order, rho, delta):
    """Brute force: replay the order on a status map and, before each step,
    sum every remaining block's window share again with NumPy; the chosen
    block must hold the largest share, and no raster-earlier block a larger
    one (near-ties within 1e-8 are left to the oracle's exact integers)."""
    y, x, c, owner = O.plan(mask, cls)
    H, W = mask.shape
    n = len(y)
    status = mask.astype(np.uint8).copy()  # 0 known, 1 lost, 2 recon
    tabs = {}
    for (B, b, _) in cls:
        tabs[B + 2 * b] = _weights(B + 2 * b, rho, delta)
    left = np.ones(n, bool)
    for step, k in enumerate(order):
        share = np.full(n, -1.0)
        for i in np.nonzero(left)[0]:
            B, b, _ = cls[c[i]]
            M = B + 2 * b
            wk, wr = tabs[M]
            y0, x0 = y[i] - b, x[i] - b
            st = np.full((M, M), 1, np.uint8)  # off-image: no weight
            ys, xs = max(0, y0), max(0, x0)
            ye, xe = min(H, y0 + M), min(W, x0 + M)
            st[ys - y0:ye - y0, xs - x0:xe - x0] = status[ys:ye, xs:xe]
            share[i] = (wk[st == 0].sum() + wr[st == 2].sum()) / wk.sum()
        top = share.max()
        assert left[k], (step, k)
        assert share[k] >= top * (1 - 1e-8), (step, k, share[k], top)
        earlier_better = [i for i in range(k) if left[i] and share[i] > share[k] * (1 + 1e-8)]
        assert not earlier_better, (step, k, earlier_better)
        left[k] = False
        status[owner == k] = 2


@pytest.mark.parametrize("seed", range(4))
def test_rule_by_brute_force(seed):
    rng = np.random.default_rng(700 + seed)
    W, H = int(rng.integers(40, 97)), int(rng.integers(40, 81))
    if seed % 2 == 0:
        cls = ((4, 14, 1),)
        mask = synth.mask_blocks_and_pixels(W, H, 4, 0.3, 0.01, seed=710 + seed)
        mask[H // 3:H // 3 + 12, W // 4:W // 4 + 16] = 1  # a larger hole
    else:
        cls = ((8, 28, 1), (4, 14, 1))
        mask = synth.mask_blocks(W, H, 8, 0.15, seed=720 + seed) | synth.mask_blocks_and_pixels(
            W, H, 4, 0.1, 0.01, seed=730 + seed)
    rho, delta = (0.8, 0.5) if seed < 2 else (0.9, 0.7)
    order = O.priority_order(mask, cls, rho=rho, delta=delta)
    assert sorted(order.tolist()) == list(range(len(order)))
    _check_rule(mask, cls, order, rho, delta)


def test_order_respecting_its_dependencies_is_bitwise_equal():
    # process by (dependency level, rank) of the optimised order's DAG: the
    # image equals the one processed in the optimised order itself
    img = synth.synth_image(96, 80, seed=41)
    mask = synth.mask_blocks_and_pixels(96, 80, 4, 0.3, 0.01, seed=42)
    mask[20:36, 30:50] = 1
    cls = ((4, 14, 30),)
    order = O.priority_order(mask, cls)
    a = O.image(img, mask, cls, order=order)
    preds = O.dependencies(mask, cls, order=order)
    lv = O.levels(preds, order=order)
    rank = np.argsort(order)
    relaxed = sorted(range(len(order)), key=lambda i: (lv[i], -rank[i]))
    # (within a level the rank is reversed on purpose: the blocks of one level
    # do not interact)
    b = O.image(img, mask, cls, order=np.array(relaxed, np.int32))
    assert np.array_equal(a, b)
    assert lv.max() < len(order) - 1
    # raster order gives a different image: the order matters
    assert not np.array_equal(a, O.image(img, mask, cls))


PLANTED = [
    ("no status update after a step", "hand",
     "                if (owner[(size_t)y * W + x] == best) status[(size_t)y * W + x] = ST_RECON;\n",
     "                if (owner[(size_t)y * W + x] == best) status[(size_t)y * W + x] = ST_LOST;\n"),
    ("ties to the raster-later block", "hand",
     "            if (best < 0 || (u128)share[i] * (u128)full[bc[best]] > (u128)share[best] * (u128)full[bc[i]])\n",
     "            if (best < 0 || (u128)share[i] * (u128)full[bc[best]] >= (u128)share[best] * (u128)full[bc[i]])\n"),
    ("reconstructed pixels at full weight", "brute",
     "    if (recon) wt = delta * wt;\n",
     "    (void)recon;\n"),
    ("smallest share first", "hand",
     "            if (best < 0 || (u128)share[i] * (u128)full[bc[best]] > (u128)share[best] * (u128)full[bc[i]])\n",
     "            if (best < 0 || (u128)share[i] * (u128)full[bc[best]] < (u128)share[best] * (u128)full[bc[i]])\n"),
]


@pytest.mark.parametrize("name,pin,old,new", PLANTED, ids=[p[0] for p in PLANTED])
def test_order_pins_reject_a_planted_mistake(name, pin, old, new, tmp_path):
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, f"planted mistake '{name}' no longer applies"
    (tmp_path / "variant.c").write_text(src.replace(old, new))
    so = str(tmp_path / "libvariant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", so, str(tmp_path / "variant.c"), "-lm"])
    with O.variant(so):
        if pin == "hand":
            assert _hand_pin()[:6] != [(0, 0), (0, 9), (9, 0), (9, 9), (0, 1), (1, 0)], name
        else:
            mask = synth.mask_blocks_and_pixels(64, 56, 4, 0.3, 0.01, seed=712)
            mask[18:30, 16:32] = 1
            cls = ((4, 14, 1),)
            order = O.priority_order(mask, cls)
            with pytest.raises(AssertionError):
                _check_rule(mask, cls, order, 0.8, 0.5)
    test_square_hole_by_hand()
