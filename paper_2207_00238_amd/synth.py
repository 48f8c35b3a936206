"""Seeded synthetic inputs for Frequency Selective Extrapolation (FSE).

This module only draws pseudo-random test images, loss masks and request
arrival traces.  It holds none of the extrapolation arithmetic, so both the
CPU reference under ``oracle/`` and the HIP path can be fed from it without
sharing any code of the method itself.

The paper evaluates on three 6024x4024 photographs and two loss masks (Sec. IV,
14 % and 62 % lost pixels) that are not distributed with it.  The images drawn
here stand in for them: a smooth gradient plus six oriented sinusoids plus
Gaussian noise, clipped to the 8-bit range and stored as float32.  The masks
mark lost pixels with 1 and known pixels with 0 (uint8).

All generators take an explicit seed and use numpy's PCG64 through
``numpy.random.default_rng``; image, mask and arrival draws use separate
seeds so that any one of them can be changed alone.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "synth_image",
    "mask_blocks",
    "mask_blocks_and_pixels",
    "mask_mixed",
    "Workload",
    "workload",
    "poisson_trace",
]


def synth_image(width: int, height: int, seed: int, period_max: float = 64.0,
                period_min: float = 4.0, n_sines: int = 6, noise_sigma: float = 2.0) -> np.ndarray:
    """Return a (height, width) float32 image with values in [0, 255].

    base 128 + linear gradient (slopes U(-40, 40) over the normalised axes)
    + ``n_sines`` sinusoids (amplitude U(20, 60), period log-uniform in
    [period_min, period_max], orientation U(0, pi), phase U(0, 2 pi))
    + N(0, noise_sigma^2), clipped to [0, 255].
    """
    rng = np.random.default_rng(seed)
    y = np.arange(height, dtype=np.float64)[:, None]
    x = np.arange(width, dtype=np.float64)[None, :]
    gx, gy = rng.uniform(-40.0, 40.0, size=2)
    xn = x / max(width - 1, 1) - 0.5
    yn = y / max(height - 1, 1) - 0.5
    img = 128.0 + gx * xn + gy * yn
    for _ in range(n_sines):
        amp = rng.uniform(20.0, 60.0)
        period = math.exp(rng.uniform(math.log(period_min), math.log(period_max)))
        theta = rng.uniform(0.0, math.pi)
        phase = rng.uniform(0.0, 2.0 * math.pi)
        img = img + amp * np.sin(2.0 * math.pi * (x * math.cos(theta) + y * math.sin(theta)) / period + phase)
    img = img + rng.normal(0.0, noise_sigma, size=(height, width))
    return np.clip(img, 0.0, 255.0).astype(np.float32)


def mask_blocks(width: int, height: int, block: int, fraction: float, seed: int) -> np.ndarray:
    """Mark round(fraction * n_blocks) whole block x block cells of the aligned
    grid as lost, chosen uniformly without replacement."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((height, width), dtype=np.uint8)
    _mark_blocks(mask, block, fraction, rng)
    return mask


def _mark_blocks(mask: np.ndarray, block: int, fraction: float, rng) -> None:
    height, width = mask.shape
    by, bx = height // block, width // block
    n = by * bx
    k = int(round(fraction * n))
    pick = rng.choice(n, size=k, replace=False)
    for idx in pick:
        r, c = divmod(int(idx), bx)
        mask[r * block:(r + 1) * block, c * block:(c + 1) * block] = 1


def mask_blocks_and_pixels(width: int, height: int, block: int, block_fraction: float,
                           pixel_fraction: float, seed: int) -> np.ndarray:
    """Lost aligned blocks plus isolated defect pixels.

    round(block_fraction * n_blocks) grid blocks are lost; then
    round(pixel_fraction * width * height) further pixels are drawn uniformly
    without replacement among the pixels that are still known.
    """
    rng = np.random.default_rng(seed)
    mask = np.zeros((height, width), dtype=np.uint8)
    _mark_blocks(mask, block, block_fraction, rng)
    known = np.flatnonzero(mask.ravel() == 0)
    k = int(round(pixel_fraction * width * height))
    pick = rng.choice(known.size, size=k, replace=False)
    mask.ravel()[known[pick]] = 1
    return mask


def mask_mixed(width: int, height: int, seed: int, frac8: float = 0.10, frac16: float = 0.05,
               row_fraction: float = 0.005) -> np.ndarray:
    """Mixed losses: 8-aligned 8x8 blocks, 16-aligned 16x16 blocks and
    full-width one-pixel-high row defects (round(row_fraction * height) rows)."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((height, width), dtype=np.uint8)
    _mark_blocks(mask, 8, frac8, rng)
    _mark_blocks(mask, 16, frac16, rng)
    nrows = int(round(row_fraction * height))
    rows = rng.choice(height, size=nrows, replace=False)
    mask[rows, :] = 1
    return mask


@dataclass(frozen=True)
class Workload:
    name: str
    image: np.ndarray
    mask: np.ndarray
    classes: tuple  # ((B, border, K), ...) largest first
    rho: float = 0.8
    gamma: float = 0.5
    recon_weight: float = 0.5


def workload(name: str, index: int = 0) -> Workload:
    """Named workloads.

    ``small``  : 128x128, sinusoid periods 4-64 px, 20 % of 4x4 blocks lost,
                 border 14 (32x32 support), K = 100.  Seeds 1 / 2.
    ``hd``     : image ``index`` of a set of 1920x1080 frames, periods 4-256 px,
                 25 % of 4x4 blocks lost plus 1 % isolated defect pixels,
                 border 14, K = 100.  Seeds 11 + 2 i / 12 + 2 i.
    ``uhd``    : image ``index`` of a set of 3840x2160 frames with mixed
                 8x8 (10 %), 16x16 (5 %) and row (0.5 %) losses; 8x8 and
                 16x16 losses use a 64x64 support with K = 200, the rest
                 4x4 blocks with a 32x32 support and K = 100.
                 Seeds 21 + 2 i / 22 + 2 i.
    """
    if name == "small":
        img = synth_image(128, 128, seed=1, period_max=64.0)
        msk = mask_blocks(128, 128, 4, 0.20, seed=2)
        return Workload(name, img, msk, ((4, 14, 100),))
    if name == "hd":
        img = synth_image(1920, 1080, seed=11 + 2 * index, period_max=256.0)
        msk = mask_blocks_and_pixels(1920, 1080, 4, 0.25, 0.01, seed=12 + 2 * index)
        return Workload(name, img, msk, ((4, 14, 100),))
    if name == "uhd":
        img = synth_image(3840, 2160, seed=21 + 2 * index, period_max=256.0)
        msk = mask_mixed(3840, 2160, seed=22 + 2 * index)
        return Workload(name, img, msk, ((16, 24, 200), (8, 28, 200), (4, 14, 100)))
    raise ValueError(f"unknown workload {name!r}")


def poisson_trace(rate_hz: float, duration_s: float, seed: int,
                  sides=(512, 1024, 2048, 4096)) -> list:
    """Request arrivals: exponential inter-arrival times at ``rate_hz`` over
    ``duration_s``; each request draws a square side from ``sides`` and a mask
    kind ('blocks' = 20 % 4x4 blocks, or 'blocks+pixels' = 25 % blocks + 1 %
    pixels) with probability 1/2 each, plus per-request image and mask seeds.
    Returns a list of dicts with keys t, side, kind, image_seed, mask_seed."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        side = int(sides[rng.integers(len(sides))])
        kind = "blocks" if rng.random() < 0.5 else "blocks+pixels"
        out.append({"t": t, "side": side, "kind": kind,
                    "image_seed": 1000 + 2 * i, "mask_seed": 1001 + 2 * i})
        i += 1
    return out


def request_inputs(req: dict):
    """Image and mask for one request of :func:`poisson_trace`."""
    side = req["side"]
    img = synth_image(side, side, seed=req["image_seed"], period_max=256.0)
    if req["kind"] == "blocks":
        msk = mask_blocks(side, side, 4, 0.20, seed=req["mask_seed"])
    else:
        msk = mask_blocks_and_pixels(side, side, 4, 0.25, 0.01, seed=req["mask_seed"])
    return img, msk
