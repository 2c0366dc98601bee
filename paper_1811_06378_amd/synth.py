"""Seeded synthetic images for the FHT workloads.

The paper runs no experiment on a dataset, so every input is synthetic: sparse
noise or dense positive values with planted straight lines, the structure a
Hough transform is meant to find.  This module holds none of the transform's
arithmetic; it only draws numbers and rasterises lines, and it is shared by the
tests, the benchmark and the smoke check.

Workloads (names used throughout):
  binary256     256 x 256 uint8, Bernoulli(0.05) {0,1} + 3 lines of slope in
                [0, 1] (mostly vertical, positive shift) set to 1.
  sparse1024    1024 x 1024 uint8, 2% of pixels uniform 0..255 + 8 lines of
                random direction set to 255.
  dense4096     4096 x 4096 float32, i.i.d. Exp(1) + 16 lines with +20.
  batch512      512 uint8 images, sides uniform in 64..2048 (independent),
                Bernoulli(0.03) + 1..4 lines of intensity 1.
  normal1024    16 x 1024 x 1024 float32 N(0,1) images, a U[0,1] weight map of
                the Hough shape, and int32 images uniform in -1000..1000.
"""
from __future__ import annotations

import numpy as np


def rng_for(name: str, seed: int = 0, index: int = 0) -> np.random.Generator:
    """Independent stream per (workload name, seed, index)."""
    key = [seed, index] + [ord(c) for c in name]
    return np.random.default_rng(np.random.SeedSequence(key))


def _draw_line_steep(img, rng, slope, value, add):
    """Rasterise x = round(x0 + slope*y) for all rows, x0 so the line crosses.
    Returns the line as (a point on it, its direction): ((x0, 0), (slope, 1))."""
    h, w = img.shape
    lo = min(0.0, -slope * (h - 1))
    hi = max(w - 1.0, w - 1.0 - slope * (h - 1))
    x0 = rng.uniform(lo, hi)
    ys = np.arange(h)
    xs = np.rint(x0 + slope * ys).astype(np.int64)
    ok = (xs >= 0) & (xs < w)
    if add:
        img[ys[ok], xs[ok]] += value
    else:
        img[ys[ok], xs[ok]] = value
    return dict(point=(float(x0), 0.0), direction=(float(slope), 1.0), pixels=int(ok.sum()))


def _draw_line_any(img, rng, value, add):
    """A line of uniform direction in [0, 180) through a uniform pixel,
    rasterised one pixel per step along its major axis."""
    h, w = img.shape
    theta = rng.uniform(0.0, np.pi)
    py, px = rng.integers(0, h), rng.integers(0, w)
    dy, dx = np.sin(theta), np.cos(theta)
    if abs(dx) >= abs(dy):               # mostly horizontal: one pixel per column
        xs = np.arange(w)
        ys = np.rint(py + (xs - px) * dy / dx).astype(np.int64)
    else:                                # mostly vertical: one pixel per row
        ys = np.arange(h)
        xs = np.rint(px + (ys - py) * dx / dy).astype(np.int64)
    ok = (xs >= 0) & (xs < w) & (ys >= 0) & (ys < h)
    if add:
        img[ys[ok], xs[ok]] += value
    else:
        img[ys[ok], xs[ok]] = value
    return dict(point=(float(px), float(py)), direction=(float(dx), float(dy)), pixels=int(ok.sum()))


# With with_lines=True the workload generators also return the planted lines
# (a point on each line, its direction and the number of pixels drawn), the
# ground truth a line detector is checked against.  The random draws are the
# same either way.

def binary256(seed: int = 0, size: int = 256, with_lines: bool = False):
    rng = rng_for("binary256", seed)
    img = (rng.random((size, size)) < 0.05).astype(np.uint8)
    lines = [_draw_line_steep(img, rng, rng.uniform(0.0, 1.0), 1, add=False) for _ in range(3)]
    return (img, lines) if with_lines else img


def sparse1024(seed: int = 0, size: int = 1024, with_lines: bool = False):
    rng = rng_for("sparse1024", seed)
    img = np.zeros((size, size), dtype=np.uint8)
    mask = rng.random((size, size)) < 0.02
    img[mask] = rng.integers(0, 256, size=int(mask.sum()), dtype=np.uint8)
    lines = [_draw_line_any(img, rng, 255, add=False) for _ in range(8)]
    return (img, lines) if with_lines else img


def dense4096(seed: int = 0, size: int = 4096, with_lines: bool = False):
    rng = rng_for("dense4096", seed)
    img = rng.standard_exponential((size, size), dtype=np.float32)
    lines = [_draw_line_any(img, rng, np.float32(20.0), add=True) for _ in range(16)]
    return (img, lines) if with_lines else img


def batch_sizes(seed: int = 0, count: int = 512, lo: int = 64, hi: int = 2048):
    rng = rng_for("batch512-sizes", seed)
    hs = rng.integers(lo, hi + 1, size=count)
    ws = rng.integers(lo, hi + 1, size=count)
    return [(int(h), int(w)) for h, w in zip(hs, ws)]


def batch_image(seed: int, index: int, h: int, w: int) -> np.ndarray:
    rng = rng_for("batch512", seed, index)
    img = (rng.random((h, w)) < 0.03).astype(np.uint8)
    for _ in range(int(rng.integers(1, 5))):
        _draw_line_any(img, rng, 1, add=False)
    return img


def batch512(seed: int = 0, count: int = 512, lo: int = 64, hi: int = 2048):
    return [batch_image(seed, i, h, w) for i, (h, w) in enumerate(batch_sizes(seed, count, lo, hi))]


def normal1024(seed: int = 0, batch: int = 16, size: int = 1024) -> np.ndarray:
    rng = rng_for("normal1024", seed)
    return rng.standard_normal((batch, size, size), dtype=np.float32)


def weight_map(shape, seed: int = 0) -> np.ndarray:
    rng = rng_for("normal1024-weight", seed)
    return rng.random(shape, dtype=np.float32)


def int_image(h: int, w: int, seed: int = 0, lo: int = -1000, hi: int = 1000) -> np.ndarray:
    rng = rng_for("int-image", seed)
    return rng.integers(lo, hi + 1, size=(h, w), dtype=np.int32)


def random_image(h: int, w: int, kind: str, seed: int = 0) -> np.ndarray:
    """Small generic images for parity sweeps: 'u8', 'i32' or 'f32'."""
    rng = rng_for("random-" + kind, seed, h * 100003 + w)
    if kind == "u8":
        return rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    if kind == "i32":
        return rng.integers(-1000, 1001, size=(h, w), dtype=np.int32)
    if kind == "f32":
        return rng.standard_exponential((h, w), dtype=np.float32)
    raise ValueError(kind)
