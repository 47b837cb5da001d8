"""Seeded synthetic inputs for the Canny workloads.

This module only draws pixels.  It holds none of the edge detector's
arithmetic, so both the oracle's tests and the GPU path can take their inputs
from it without sharing any part of the method.

The paper tests on an unpublished "set of images" (Section 2.2) and on
application images from several disciplines (Fig. 7); neither is available.
These generators stand in for them with images whose structure drives the
method the same way: smooth shading (weak gradients), step edges of varied
contrast and orientation (rectangles and disks), and sensor-like noise.

Recipes (all draws come from ``numpy.random.default_rng(seed)`` in the order
listed, so an image is a pure function of its size and seed):

``natural_u8(H, W, seed)``
  1. background: value noise on a lattice of period 64 px, lattice values
     U[0, 255), bilinear interpolation with smoothstep weights 3t^2 - 2t^3;
  2. 40 shapes painted in order, each a rectangle or a disk (p = 1/2), offset
     sign*c from the background with c ~ U{30..120}, sign = +-1; later shapes
     overwrite earlier ones; rectangle sides ~ U{8..max(8, min(H,W)/4)},
     disk radius ~ U{4..max(4, min(H,W)/8)}, positions uniform;
  3. i.i.d. Gaussian noise N(0, 8^2), rounded half-to-even, clipped to 0..255.

``spiral_u8(N, seed, noise_sigma)``
  flat 96 background, a rectangular spiral of one-pixel line with arm
  spacing 8 and contrast 56 whose first 16 pixels have contrast 120 (the only
  strong seed), plus the Gaussian noise of step 3 at ``noise_sigma``.

``batch_shapes(n, seed)``
  n (H, W) pairs with H ~ U{240..2160} and W ~ U{320..3840}.
"""
from __future__ import annotations

import numpy as np

PERIOD = 64
N_SHAPES = 40
NOISE_SIGMA = 8.0
CHUNK_ROWS = 1024


def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def _value_noise(rng, H, W):
    gh = -(-H // PERIOD) + 2
    gw = -(-W // PERIOD) + 2
    lat = rng.uniform(0.0, 255.0, size=(gh, gw))
    xs = np.arange(W) / PERIOD
    ix = np.floor(xs).astype(np.int64)
    wx = _smoothstep(xs - ix)
    out = np.empty((H, W), dtype=np.float32)
    for y0 in range(0, H, CHUNK_ROWS):
        y1 = min(H, y0 + CHUNK_ROWS)
        ys = np.arange(y0, y1) / PERIOD
        iy = np.floor(ys).astype(np.int64)
        wy = _smoothstep(ys - iy)[:, None]
        top = lat[iy][:, ix] * (1.0 - wx) + lat[iy][:, ix + 1] * wx
        bot = lat[iy + 1][:, ix] * (1.0 - wx) + lat[iy + 1][:, ix + 1] * wx
        out[y0:y1] = top * (1.0 - wy) + bot * wy
    return out


def _paint_shapes(rng, H, W, off):
    m = min(H, W)
    for _ in range(N_SHAPES):
        kind = int(rng.integers(2))
        c = int(rng.integers(30, 121))
        sign = 1 if rng.integers(2) else -1
        if kind == 0:
            hmax = max(8, m // 4)
            h = int(rng.integers(8, hmax + 1))
            w = int(rng.integers(8, hmax + 1))
            y0 = int(rng.integers(0, max(1, H - h + 1)))
            x0 = int(rng.integers(0, max(1, W - w + 1)))
            off[y0:y0 + h, x0:x0 + w] = sign * c
        else:
            rmax = max(4, m // 8)
            r = int(rng.integers(4, rmax + 1))
            cy = int(rng.integers(0, H))
            cx = int(rng.integers(0, W))
            ya, yb = max(0, cy - r), min(H, cy + r + 1)
            xa, xb = max(0, cx - r), min(W, cx + r + 1)
            yy = np.arange(ya, yb)[:, None] - cy
            xx = np.arange(xa, xb)[None, :] - cx
            inside = yy * yy + xx * xx <= r * r
            sub = off[ya:yb, xa:xb]
            sub[inside] = sign * c


def _add_noise_clip(rng, img_f32, sigma):
    H, W = img_f32.shape
    out = np.empty((H, W), dtype=np.uint8)
    for y0 in range(0, H, CHUNK_ROWS):
        y1 = min(H, y0 + CHUNK_ROWS)
        v = img_f32[y0:y1].astype(np.float64)
        if sigma > 0:
            v = v + rng.normal(0.0, sigma, size=v.shape)
        out[y0:y1] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return out


def natural_u8(H: int, W: int, seed: int) -> np.ndarray:
    """Shaded background + 40 step-edged shapes + noise, uint8 (H, W)."""
    rng = np.random.default_rng(seed)
    bg = _value_noise(rng, H, W)
    off = np.zeros((H, W), dtype=np.float32)
    _paint_shapes(rng, H, W, off)
    bg += off
    return _add_noise_clip(rng, bg, NOISE_SIGMA)


def natural_unit_f32(H: int, W: int, seed: int) -> np.ndarray:
    """``natural_u8`` scaled to [0, 1] as float32."""
    return natural_u8(H, W, seed).astype(np.float32) / np.float32(255.0)


def spiral_path(N: int, spacing: int = 8, margin: int = 4):
    """Pixel coordinates (ys, xs) of a clockwise rectangular spiral, outside in."""
    ys, xs = [], []
    top, left, bottom, right = margin, margin, N - 1 - margin, N - 1 - margin
    while top <= bottom and left <= right:
        ys.append(np.full(right - left + 1, top)); xs.append(np.arange(left, right + 1))
        if bottom - top < 1:
            break
        ys.append(np.arange(top + 1, bottom + 1)); xs.append(np.full(bottom - top, right))
        if right - left < 1:
            break
        ys.append(np.full(right - left, bottom)); xs.append(np.arange(right - 1, left - 1, -1))
        up_end = top + spacing
        if bottom - 1 < up_end:
            break
        ys.append(np.arange(bottom - 1, up_end - 1, -1)); xs.append(np.full(bottom - up_end, left))
        if left + spacing > right - spacing:
            break
        ys.append(np.full(spacing, up_end)); xs.append(np.arange(left + 1, left + spacing + 1))
        top, left, bottom, right = up_end, left + spacing, bottom - spacing, right - spacing
    return np.concatenate(ys).astype(np.int64), np.concatenate(xs).astype(np.int64)


def spiral_u8(N: int, seed: int, noise_sigma: float = NOISE_SIGMA,
              contrast: int = 56, seed_contrast: int = 120, seed_len: int = 16) -> np.ndarray:
    """One long weak-edge spiral seeded by a single short strong segment."""
    rng = np.random.default_rng(seed)
    img = np.full((N, N), 96.0, dtype=np.float32)
    ys, xs = spiral_path(N)
    img[ys, xs] = 96.0 + contrast
    img[ys[:seed_len], xs[:seed_len]] = 96.0 + seed_contrast
    return _add_noise_clip(rng, img, noise_sigma)


def batch_shapes(n: int = 256, seed: int = 3):
    rng = np.random.default_rng(seed)
    H = rng.integers(240, 2161, size=n)
    W = rng.integers(320, 3841, size=n)
    return [(int(h), int(w)) for h, w in zip(H, W)]


def sigma_init(n: int = 32, seed: int = 4, lo: float = 1.0, hi: float = 3.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n).astype(np.float32)


def random_classes(H: int, W: int, seed: int, p_weak: float, p_strong: float) -> np.ndarray:
    """i.i.d. class map (0 none, 1 weak, 2 strong) for hysteresis-only tests."""
    u = np.random.default_rng(seed).random((H, W))
    c = np.zeros((H, W), dtype=np.uint8)
    c[u < p_weak + p_strong] = 1
    c[u < p_strong] = 2
    return c
