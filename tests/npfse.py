"""Brute-force NumPy model of one FSE block -- a checker of the oracle (test
infrastructure).

Written from the block model of Sec. II and the readings R6, R7, R9-R12,
independently of ``oracle/fse_oracle.c``: no code, table or loop structure
is shared.

* Weights (R6, R7): isotropic decay rho^dist from the window centre
  ((M-1)/2, (M-1)/2); a known pixel has weight rho^dist, a reconstructed one
  delta rho^dist, a lost or off-image pixel 0.
* Greedy fit (R9-R11): the residual is kept in the pixel domain; before every
  step its weighted spectrum is recomputed from scratch with the textbook
  ``numpy.fft.fft2`` (the oracle updates its spectrum in place instead); the
  first maximiser of |R|^2 is chosen, alpha = gamma R[u, v] / W0, and the
  residual loses alpha times the basis function e^{+2 pi i (u m + v n) / M}.
* Synthesis (R12): Re of the sum of alpha e^{+2 pi i (u m + v n) / M} at the
  block's pixels, the phase evaluated in floating point (no integer phase
  table).

Slow (one FFT per step) and meant for single blocks.
"""
from __future__ import annotations

import numpy as np

KNOWN, LOST, RECON = 0, 1, 2


def weights(status_win, M: int, rho: float, delta: float):
    """Weights of an M x M window; status_win holds KNOWN, LOST, RECON or -1
    (off the image)."""
    c = (M - 1) / 2.0
    mm, nn = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    decay = rho ** np.hypot(mm - c, nn - c)
    return np.where(status_win == KNOWN, decay, np.where(status_win == RECON, delta * decay, 0.0))


def basis(M: int, u: int, v: int):
    mm, nn = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    return np.exp(2j * np.pi * (u * mm + v * nn) / M)


def fit(s, w, K: int, gamma: float):
    """Greedy sparse fit; returns (chosen flat indices, coefficients, W0)."""
    M = s.shape[0]
    W0 = float(w.sum())
    r = np.where(w > 0, s, 0.0).astype(complex)
    sel, alpha = [], []
    if W0 <= 0:
        return sel, alpha, W0
    for _ in range(K):
        R = np.fft.fft2(w * r)
        q = int(np.argmax(np.abs(R) ** 2))  # first maximiser
        u, v = divmod(q, M)
        a = gamma * R[u, v] / W0
        r = r - a * basis(M, u, v)
        sel.append(q)
        alpha.append(a)
    return sel, alpha, W0


def synth(sel, alpha, M: int, rows, cols):
    """Re of the model at window positions (rows[i], cols[j])."""
    g = np.zeros((len(rows), len(cols)), complex)
    for q, a in zip(sel, alpha):
        u, v = divmod(q, M)
        g += a * np.exp(2j * np.pi * (u * np.asarray(rows)[:, None] + v * np.asarray(cols)[None, :]) / M)
    return g.real


def one_block(val, status, y0: int, x0: int, B: int, b: int, K: int, rho=0.8, gamma=0.5, delta=0.5):
    """The block of edge B at (y0, x0) with support border b, extrapolated
    from the image state (val, status).  Returns (B x B model values, chosen
    indices, W0)."""
    H, W = val.shape
    M = B + 2 * b
    ys = np.arange(y0 - b, y0 - b + M)
    xs = np.arange(x0 - b, x0 - b + M)
    inside = (ys[:, None] >= 0) & (ys[:, None] < H) & (xs[None, :] >= 0) & (xs[None, :] < W)
    yc = np.clip(ys, 0, H - 1)
    xc = np.clip(xs, 0, W - 1)
    st = np.where(inside, status[np.ix_(yc, xc)], -1)
    w = weights(st, M, rho, delta)
    s = np.where(w > 0, val[np.ix_(yc, xc)], 0.0)
    sel, alpha, W0 = fit(s, w, K, gamma)
    core = np.arange(b, b + B)
    return synth(sel, alpha, M, core, core), np.array(sel, np.int64), W0


def plan(mask, classes):
    """Processing blocks (y0, x0, class) in raster order and the owner of
    every lost pixel (R2): each class but the last takes the aligned squares
    of its edge that are entirely lost (inside the image) and not taken by a
    larger class; the last class takes every aligned cell, clipped at the
    image edge, that still holds a lost pixel of its own."""
    H, W = mask.shape
    owner_of = -np.ones((H, W), np.int64)
    found = []
    for c, (B, _, _) in enumerate(classes):
        last = c == len(classes) - 1
        for y0 in range(0, H, B):
            for x0 in range(0, W, B):
                cell = (slice(y0, min(H, y0 + B)), slice(x0, min(W, x0 + B)))
                free_lost = (mask[cell] != 0) & (owner_of[cell] < 0)
                if last:
                    take = bool(free_lost.any())
                else:
                    take = y0 + B <= H and x0 + B <= W and bool(free_lost.all())
                if take:
                    owner_of[cell][free_lost] = len(found)
                    found.append((y0, x0, c))
    order = sorted(range(len(found)), key=lambda i: (found[i][0], found[i][1]))
    rank = np.empty(len(found), np.int64)
    rank[order] = np.arange(len(found))
    owner = np.where(owner_of >= 0, rank[np.maximum(owner_of, 0)], -1)
    return [found[i] for i in order], owner


def image(img, mask, classes, rho=0.8, gamma=0.5, delta=0.5):
    """Whole image in raster order of the blocks: each block is fitted to the
    current image state and writes its own lost pixels, which then count as
    reconstructed for the blocks after it."""
    H, W = mask.shape
    blocks, owner = plan(mask, classes)
    val = np.where(mask != 0, 0.0, np.asarray(img, np.float64))
    status = np.where(mask != 0, LOST, KNOWN).astype(np.uint8)
    for i, (y0, x0, c) in enumerate(blocks):
        B, b, K = classes[c]
        model, _, _ = one_block(val, status, y0, x0, B, b, K, rho, gamma, delta)
        ys, xs = slice(y0, min(H, y0 + B)), slice(x0, min(W, x0 + B))
        mine = owner[ys, xs] == i
        val[ys, xs][mine] = model[:ys.stop - y0, :xs.stop - x0][mine]
        status[ys, xs][mine] = RECON
    return val
