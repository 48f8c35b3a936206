"""Python face of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

Contents
  * ctypes access to ``fse_oracle.c`` (FP64 Frequency Selective
    Extrapolation, Sec. II of the paper): :func:`image`, :func:`block`,
    :func:`plan`, and :func:`image_levels` (the same result with the blocks
    of each dependency level run in parallel on the host's cores).
  * :func:`tiling` -- the paper's compact tiling, Algorithm 1 with
    eqs. (1)-(5), written from the equations in pure Python integers.
  * :func:`tiles_with_stripe` and :func:`image_tiled` -- the overlapping-tile
    framework of Sec. III: every tile grown by a stripe of d pixels on each
    side, processed as an independent image, cropped back to its core and
    merged.
  * :func:`dependencies` -- which earlier blocks a block must see finished in
    raster order or in a given processing order (a block reads the pixels of
    its support window, and writes its own lost pixels).
  * :func:`priority_order` -- the optimised processing order (Sec. II),
    reading R17.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fse_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
TOPN = 4

_lib = None


def build(force: bool = False) -> str:
    """Compile fse_oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


class variant:
    """Context manager: the functions of this module run on another build of
    the oracle's C code (a library at ``path``) until the block exits.  The
    tests use it to show that the pins reject an oracle with a planted
    mistake."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = _lib
        _lib = _bind(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def _bind(lib):
    P = ctypes.POINTER
    d, i, u8 = ctypes.c_double, ctypes.c_int, ctypes.c_uint8
    lib.fse_oracle_block.restype = d
    lib.fse_oracle_block.argtypes = [i, P(d), P(d), P(d), i, d, P(i), P(d), P(d), P(d), P(d), P(i)]
    lib.fse_oracle_plan.restype = i
    lib.fse_oracle_plan.argtypes = [P(u8), i, i, P(i), i, P(i), P(i), P(i), i, P(i)]
    lib.fse_oracle_one_block.restype = d
    lib.fse_oracle_one_block.argtypes = [P(d), P(u8), i, i, i, i, i, i, i, d, d, d, P(d), P(i)]
    lib.fse_oracle_priority_order.restype = i
    lib.fse_oracle_priority_order.argtypes = [P(u8), i, i, P(i), i, d, d, P(i)]
    lib.fse_oracle_image_levels.restype = i
    lib.fse_oracle_image_levels.argtypes = [P(d), P(u8), i, i, P(i), i, d, d, d, P(d), P(i), P(i)]
    lib.fse_oracle_image.restype = i
    lib.fse_oracle_image.argtypes = [P(d), P(u8), i, i, P(i), i, d, d, d, P(i), P(d), i, P(i), P(d),
                                     P(i), P(d), P(d)]
    return lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def block(s, w, K: int, gamma: float, history: bool = False):
    """Greedy sparse fit of one M x M window (complex or real ``s``, weights
    ``w``).  Returns dict(W0, sel, alpha (complex K), e_top, i_top[, R])."""
    lib = _load()
    s = np.asarray(s)
    M = s.shape[0]
    sr = np.ascontiguousarray(s.real, dtype=np.float64)
    si = np.ascontiguousarray(s.imag, dtype=np.float64) if np.iscomplexobj(s) else None
    w = np.ascontiguousarray(w, dtype=np.float64)
    sel = np.zeros(K, np.int32)
    ar = np.zeros(K)
    ai = np.zeros(K)
    et = np.zeros(K * TOPN)
    it = np.zeros(K * TOPN, np.int32)
    hist = np.zeros((K + 1) * 2 * M * M) if history else None
    W0 = lib.fse_oracle_block(M, _p(sr, ctypes.c_double), _p(si, ctypes.c_double), _p(w, ctypes.c_double),
                              K, gamma, _p(sel, ctypes.c_int), _p(ar, ctypes.c_double),
                              _p(ai, ctypes.c_double), _p(hist, ctypes.c_double), _p(et, ctypes.c_double),
                              _p(it, ctypes.c_int))
    out = {"W0": W0, "sel": sel, "alpha": ar + 1j * ai, "e_top": et.reshape(K, TOPN),
           "i_top": it.reshape(K, TOPN)}
    if history:
        h = hist.reshape(K + 1, 2, M, M)
        out["R"] = h[:, 0] + 1j * h[:, 1]
    return out


def one_block(val, status, y0, x0, B, b, K, rho=0.8, gamma=0.5, delta=0.5):
    """Extrapolate one block from a given image state: ``val`` (H, W) values,
    ``status`` (H, W) uint8 with 0 known, 1 lost, 2 reconstructed.  Returns
    (values of the model at the B x B block pixels, selected indices, W0)."""
    lib = _load()
    val = np.ascontiguousarray(val, dtype=np.float64)
    status = np.ascontiguousarray(status, dtype=np.uint8)
    H, W = val.shape
    outv = np.zeros(B * B)
    sel = np.zeros(max(K, 1), np.int32)
    W0 = lib.fse_oracle_one_block(_p(val, ctypes.c_double), _p(status, ctypes.c_uint8), W, H, y0, x0, B, b, K,
                                  rho, gamma, delta, _p(outv, ctypes.c_double), _p(sel, ctypes.c_int))
    return outv.reshape(B, B), sel[:K], W0


def _classes_arr(classes):
    return np.ascontiguousarray(np.array(classes, dtype=np.int32).reshape(-1))


def plan(mask, classes):
    """Processing blocks in raster order: arrays (y0, x0, class) and the
    owner map (block index per lost pixel, -1 elsewhere)."""
    lib = _load()
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    H, W = mask.shape
    ca = _classes_arr(classes)
    n = lib.fse_oracle_plan(_p(mask, ctypes.c_uint8), W, H, _p(ca, ctypes.c_int), len(classes), None, None,
                            None, 0, None)
    n = -n if n < 0 else n
    y = np.zeros(max(n, 1), np.int32)
    x = np.zeros(max(n, 1), np.int32)
    c = np.zeros(max(n, 1), np.int32)
    owner = np.zeros((H, W), np.int32)
    r = lib.fse_oracle_plan(_p(mask, ctypes.c_uint8), W, H, _p(ca, ctypes.c_int), len(classes), _p(y, ctypes.c_int),
                            _p(x, ctypes.c_int), _p(c, ctypes.c_int), n, _p(owner, ctypes.c_int))
    assert r == n
    return y[:n], x[:n], c[:n], owner


def priority_order(mask, classes, rho=0.8, delta=0.5):
    """Optimised processing order (Sec. II; reading R17 in fse_oracle.c): the
    raster indices of the blocks in the order they are processed, each step
    taking the remaining block whose window offers the largest share of
    usable weight (ties to the raster-earlier block)."""
    lib = _load()
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    H, W = mask.shape
    ca = _classes_arr(classes)
    n = len(plan(mask, classes)[0])
    order = np.zeros(max(n, 1), np.int32)
    r = lib.fse_oracle_priority_order(_p(mask, ctypes.c_uint8), W, H, _p(ca, ctypes.c_int), len(classes), rho,
                                      delta, _p(order, ctypes.c_int))
    if r < 0:
        raise ValueError("oracle: bad arguments")
    assert r == n
    return order[:n]


def image(img, mask, classes, rho=0.8, gamma=0.5, delta=0.5, order=None, trace=False):
    """FP64 extrapolation of a whole image.  Returns the output (float64) or,
    with ``trace=True``, (out, trace dict with sel/e_top/i_top/alpha/W0 per
    raster block)."""
    lib = _load()
    img = np.ascontiguousarray(img, dtype=np.float64)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    H, W = img.shape
    assert mask.shape == (H, W)
    ca = _classes_arr(classes)
    out = np.zeros((H, W))
    order_a = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    Kmax = max(c[2] for c in classes)
    tr = None
    if trace:
        nb, _, _, _ = plan(mask, classes)
        n = len(nb)
        tr = {"sel": np.full((n, Kmax), -1, np.int32), "e_top": np.zeros((n, Kmax, TOPN)),
              "i_top": np.full((n, Kmax, TOPN), -1, np.int32), "alpha": np.zeros((n, Kmax, 2)),
              "W0": np.zeros(n)}
    rc = lib.fse_oracle_image(_p(img, ctypes.c_double), _p(mask, ctypes.c_uint8), W, H, _p(ca, ctypes.c_int),
                              len(classes), rho, gamma, delta, _p(order_a, ctypes.c_int),
                              _p(out, ctypes.c_double), Kmax,
                              _p(tr["sel"], ctypes.c_int) if trace else None,
                              _p(tr["e_top"], ctypes.c_double) if trace else None,
                              _p(tr["i_top"], ctypes.c_int) if trace else None,
                              _p(tr["alpha"], ctypes.c_double) if trace else None,
                              _p(tr["W0"], ctypes.c_double) if trace else None)
    if rc == -1:
        raise ValueError("oracle: bad arguments")
    if trace:
        tr["alpha"] = tr["alpha"][..., 0] + 1j * tr["alpha"][..., 1]
        tr["degenerate"] = rc == -2
        return out, tr
    return out


def image_levels(img, mask, classes, rho=0.8, gamma=0.5, delta=0.5):
    """The raster-order result of :func:`image`, with the blocks of each
    dependency level run in parallel on the host's cores (OpenMP; bitwise the
    same output).  Returns (out, number of levels, threads used)."""
    lib = _load()
    img = np.ascontiguousarray(img, dtype=np.float64)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    H, W = img.shape
    ca = _classes_arr(classes)
    out = np.zeros((H, W))
    nl = ctypes.c_int(0)
    nt = ctypes.c_int(0)
    rc = lib.fse_oracle_image_levels(_p(img, ctypes.c_double), _p(mask, ctypes.c_uint8), W, H,
                                     _p(ca, ctypes.c_int), len(classes), rho, gamma, delta,
                                     _p(out, ctypes.c_double), ctypes.byref(nl), ctypes.byref(nt))
    if rc == -1:
        raise ValueError("oracle: bad arguments")
    return out, nl.value, nt.value


# ---------------------------------------------------------------------------
# Algorithm 1: compact tiling (Sec. III, eqs. (1)-(5))
# ---------------------------------------------------------------------------

def _round_half_up(q: Fraction) -> int:
    """round() of a non-negative rational, halves rounded up."""
    return int((q + Fraction(1, 2)) // 1)


def tiling(W: int, H: int, N: int):
    """Tiles (x_T, y_T, w_T, h_T) of a W x H image into N tiles, from
    eqs. (1)-(5) of Sec. III.

    Landscape is assumed (W >= H); a portrait image is tiled as its transpose.
    Each equation gives one list: eq. (1) the aspect ratio r = W / H; eq. (2)
    the number of rows n_R = max(1, round(sqrt(N / r))), the square root
    rounded exactly (round(sqrt(q)) = k iff (k - 1/2)^2 <= q < (k + 1/2)^2,
    halves up); eq. (3) the tiles n_C of every row i = 1..n_R (ceil(N / n_R)
    while i <= N mod n_R, else floor); eq. (4) the height h_T of every row,
    the last row taking what is left of H; eq. (5) the width w_T of every
    tile j = 1..n_C of a row (ceil(W / n_C) while j <= W mod n_C, else
    floor).  Offsets are the running sums of heights and widths.  For large
    N the heights of eq. (4) can add up to more than H: rows are then cut at
    the bottom edge, and rows past it are empty.
    """
    if W < H:
        return [(y, x, h, w) for (x, y, w, h) in tiling(H, W, N)]
    r = Fraction(W, H)                                           # eq. (1)
    q = Fraction(N) / r
    k = 0
    while Fraction(2 * k + 1, 2) ** 2 <= q:
        k += 1
    n_R = max(1, k)                                              # eq. (2)
    rows = range(1, n_R + 1)
    n_C = [-(-N // n_R) if i <= N % n_R else N // n_R for i in rows]      # eq. (3)
    h_T = [(H * c) // N + ((H * c) % N) // n_R for c in n_C]             # eq. (4)
    y_T = [min(H, sum(h_T[:i])) for i in range(n_R)]  # offsets, cut at the bottom edge
    h_T = [min(H, y + h) - y for y, h in zip(y_T, h_T)]
    h_T[-1] = H - y_T[-1]  # the last row takes what is left
    tiles = []
    for y, h, c in zip(y_T, h_T, n_C):
        w_T = [-(-W // c) if j <= W % c else W // c for j in range(1, c + 1)]  # eq. (5)
        x_T = [sum(w_T[:j]) for j in range(c)]
        tiles += [(x, y, w, h) for x, w in zip(x_T, w_T)]
    return tiles


def tiling_vertical(W: int, H: int, N: int):
    """The straightforward alternative the compact tiling is measured against:
    N vertical stripes of the full height, widths as in eq. (5) with all N
    tiles in one row (ceil(W / N) for the first W mod N stripes, else floor)."""
    tiles = []
    x_T = 0
    for j in range(1, N + 1):
        w_T = -(-W // N) if j <= W % N else W // N
        tiles.append((x_T, 0, w_T, H))
        x_T += w_T
    return tiles


def tiles_with_stripe(W: int, H: int, N: int, d: int, align: int = 1, vertical: bool = False):
    """Core tiles of :func:`tiling` (or of :func:`tiling_vertical`), optionally
    with every interior edge moved down to a multiple of ``align`` (block-grid
    alignment), each grown by the stripe d on all four sides and clipped to the
    image.  Returns a list of (core, extended) rectangles, each (x, y, w, h)."""
    out = []
    for (x, y, w, h) in (tiling_vertical(W, H, N) if vertical else tiling(W, H, N)):
        x1, y1 = x + w, y + h
        if align > 1:
            x0a = (x // align) * align
            y0a = (y // align) * align
            x1a = W if x1 == W else (x1 // align) * align
            y1a = H if y1 == H else (y1 // align) * align
            x, y, x1, y1 = x0a, y0a, x1a, y1a
        ex0, ey0 = max(0, x - d), max(0, y - d)
        ex1, ey1 = min(W, x1 + d), min(H, y1 + d)
        out.append(((x, y, x1 - x, y1 - y), (ex0, ey0, ex1 - ex0, ey1 - ey0)))
    return out


def image_tiled(img, mask, classes, N: int, d: int, align: int, rho=0.8, gamma=0.5, delta=0.5,
                vertical: bool = False, optimized_order: bool = False):
    """Overlapping-tile framework on the CPU: each extended tile is extrapolated
    as an independent image, cropped to its core and merged (Sec. III); with
    ``optimized_order`` each tile in its own optimised processing order."""
    H, W = img.shape
    out = np.zeros((H, W))
    for (core, ext) in tiles_with_stripe(W, H, N, d, align, vertical):
        ex, ey, ew, eh = ext
        if ew <= 0 or eh <= 0:
            continue
        sm = mask[ey:ey + eh, ex:ex + ew]
        order = priority_order(sm, classes, rho, delta) if optimized_order else None
        sub = image(img[ey:ey + eh, ex:ex + ew], sm, classes, rho, gamma, delta, order=order)
        cx, cy, cw, ch = core
        out[cy:cy + ch, cx:cx + cw] = sub[cy - ey:cy - ey + ch, cx - ex:cx - ex + cw]
    return out


# ---------------------------------------------------------------------------
# Raster-order dependencies
# ---------------------------------------------------------------------------

def dependencies(mask, classes, order=None):
    """For every raster block j, the blocks i processed before j (raster
    order, or the given processing order of raster indices) that must be
    finished before j starts so that j sees the same window as in that order:
    i owns a lost pixel inside j's support window (j reads it as
    reconstructed), or j owns a lost pixel inside i's window (i must read it
    before j writes it).  Brute force over pixels; meant for small images."""
    y, x, c, owner = plan(mask, classes)
    H, W = mask.shape
    n = len(y)
    rank = np.arange(n) if order is None else np.argsort(np.asarray(order))
    win_owners = []
    for j in range(n):
        B, b, _ = classes[c[j]]
        M = B + 2 * b
        y0, x0 = y[j] - b, x[j] - b
        sub = owner[max(0, y0):min(H, y0 + M), max(0, x0):min(W, x0 + M)]
        win_owners.append(set(int(v) for v in np.unique(sub) if v >= 0 and v != j))
    preds = [set() for _ in range(n)]
    for j in range(n):
        for i in win_owners[j]:
            a, bb = (i, j) if rank[i] < rank[j] else (j, i)
            preds[bb].add(a)
    return [sorted(p) for p in preds]


def levels(preds, order=None):
    """Longest-path level of every block (sources at level 0); blocks are
    visited in raster order or in the given processing order."""
    lv = np.zeros(len(preds), np.int64)
    for j in (range(len(preds)) if order is None else order):
        if preds[j]:
            lv[j] = 1 + max(lv[i] for i in preds[j])
    return lv
