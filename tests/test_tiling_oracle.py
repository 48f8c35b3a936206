"""Pins of the tiling oracle (Algorithm 1, eqs. (1)-(5)) against the hand
derivation of the paper's W=1024, H=480, N=22 example and against the
properties the paper asks of a tiling (Sec. III: tiles cover the image,
about equal areas, the requested count)."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiling_1024x480_n22.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    return rows


def test_worked_example():
    assert O.tiling(1024, 480, 22) == _golden()


def _cover(W, H, tiles):
    cov = np.zeros((H, W), np.int32)
    for (x, y, w, h) in tiles:
        assert w >= 0 and h >= 0
        cov[y:y + h, x:x + w] += 1
    return cov


@pytest.mark.parametrize("W,H,N", [(1920, 1080, 32), (3840, 2160, 64), (6024, 4024, 32), (128, 128, 4),
                                   (480, 1920, 7), (1000, 999, 13), (640, 64, 9), (64, 640, 9)])
def test_partition_and_count(W, H, N):
    tiles = O.tiling(W, H, N)
    assert len(tiles) == N
    cov = _cover(W, H, tiles)
    assert (cov == 1).all()


def test_row_structure_and_equal_areas():
    for W, H, N in itertools.product([640, 1024, 1920, 3840], [480, 1080, 2160], range(1, 40)):
        tiles = O.tiling(W, H, N)
        assert len(tiles) == N
        # rows run along the long side (portrait images are tiled transposed)
        ax = 1 if W >= H else 0
        Wl, Hl = max(W, H), min(W, H)
        ys = sorted(set(t[ax] for t in tiles))
        # number of rows follows eq. (2): round(sqrt(N H / W)), at least 1
        nr = max(1, int(math.floor(math.sqrt(N * Hl / Wl) + 0.5)))
        assert len(ys) == nr
        counts = [sum(1 for t in tiles if t[ax] == y) for y in ys]
        assert max(counts) - min(counts) <= 1
        assert sum(t[2] * t[3] for t in tiles) == W * H
        # requirement 1: roughly equal areas (the last row absorbs rounding)
        areas = np.array([t[2] * t[3] for t in tiles], float)
        assert areas.max() / areas.min() < 1.6


def test_portrait_swaps_axes():
    land = O.tiling(1024, 480, 22)
    port = O.tiling(480, 1024, 22)
    assert port == [(y, x, h, w) for (x, y, w, h) in land]


def test_single_tile_and_stripes():
    assert O.tiling(300, 200, 1) == [(0, 0, 300, 200)]
    # very wide image: one row of vertical stripes
    t = O.tiling(4000, 100, 5)
    assert [tt[1] for tt in t] == [0] * 5 and [tt[2] for tt in t] == [800] * 5


def test_stripe_and_alignment():
    W, H = 1920, 1080
    for (core, ext) in O.tiles_with_stripe(W, H, 16, 32, align=16):
        x, y, w, h = core
        ex, ey, ew, eh = ext
        assert x % 16 == 0 and y % 16 == 0
        assert ex == max(0, x - 32) and ey == max(0, y - 32)
        assert ex + ew == min(W, x + w + 32) and ey + eh == min(H, y + h + 32)
    cov = _cover(W, H, [c for c, _ in O.tiles_with_stripe(W, H, 16, 32, align=16)])
    assert (cov == 1).all()


@pytest.mark.parametrize("W,H,N", [(1920, 1080, 256), (1920, 1080, 1024), (3840, 2160, 4096), (640, 480, 300)])
def test_large_n_rows_clipped_still_partition(W, H, N):
    # eq. (4) overshoots H for these N; with the rows clipped at the bottom the
    # tiles still cover the image exactly once and none has a negative size
    tiles = O.tiling(W, H, N)
    assert len(tiles) == N
    assert all(t[2] >= 0 and t[3] >= 0 for t in tiles)
    cov = _cover(W, H, tiles)
    assert (cov == 1).all()


@pytest.mark.parametrize("W,H,N", [(1024, 480, 22), (37, 11, 5), (100, 300, 7), (64, 64, 64)])
def test_vertical_tiling_partition_and_widths(W, H, N):
    # N full-height stripes, widths differing by at most one pixel, the wider
    # ones first (eq. (5) with a single row)
    tiles = O.tiling_vertical(W, H, N)
    assert len(tiles) == N
    cov = _cover(W, H, tiles)
    assert (cov == 1).all()
    ws = [w for (_, _, w, _) in tiles]
    assert all(h == H and y == 0 for (_, y, _, h) in tiles)
    assert max(ws) - min(ws) <= 1 and ws == sorted(ws, reverse=True)
    assert sum(ws) == W


def test_vertical_stripes_overlap_more_than_compact():
    # the reason for the compact tiling: for the same N and d the stripes of
    # the vertical tiling cover more extra pixels (Sec. III)
    W, H, N, d = 1920, 1080, 32, 32
    def extra(tiles):
        return sum(ew * eh for (_, (ex, ey, ew, eh)) in tiles) - W * H
    assert extra(O.tiles_with_stripe(W, H, N, d, 4, vertical=True)) > 1.5 * extra(O.tiles_with_stripe(W, H, N, d, 4))
