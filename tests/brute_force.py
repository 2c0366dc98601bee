"""Brute-force Hough sums along explicitly built dyadic patterns (tiny n only).

Independent of the oracle: the pattern comes from the bitwise closed form
    D_n(s, y) = sum_j bit_{k-1-j}(y) * ((s >> j) - (s >> (j+1))),
(the same halving rule as Brady's recursion, unrolled over the bits of y),
and every Hough cell is a direct sum over the pattern's pixels, with the
padding, transposition and direction of each quadrant written from their
definitions.  O(n^2 W) per quadrant.
"""
from __future__ import annotations

import numpy as np


def pow2_ceil(v: int) -> int:
    p = 1
    while p < v:
        p *= 2
    return p


def pattern_closed_form(n: int, s: int, y: int) -> int:
    k = n.bit_length() - 1
    d = 0
    for j in range(k):
        if (y >> (k - 1 - j)) & 1:
            d += (s >> j) - (s >> (j + 1))
    return d


def pattern_table(n: int) -> np.ndarray:
    """tab[s, y] = D_n(s, y)."""
    return np.array([[pattern_closed_form(n, s, y) for y in range(n)] for s in range(n)],
                    dtype=np.int64)


def padded(img: np.ndarray, transposed: bool) -> np.ndarray:
    h, w = img.shape
    hp, wp = pow2_ceil(h), pow2_ceil(w)
    W = hp + wp
    src = img.T if transposed else img
    n = wp if transposed else hp
    out = np.zeros((n, W), dtype=np.float64)
    out[: src.shape[0], : src.shape[1]] = src
    return out


def quadrant(img: np.ndarray, q: int, reduce=np.sum) -> np.ndarray:
    """Every cell reduced directly over its pattern's pixels (np.sum, or
    np.max for the max transform)."""
    transposed = q >= 3
    sign = 1 if q in (1, 4) else -1
    src = padded(np.asarray(img, dtype=np.float64), transposed)
    n, W = src.shape
    tab = pattern_table(n)
    rows = np.arange(n)
    out = np.zeros((n, W), dtype=np.float64)
    for s in range(n):
        for x in range(W):
            cols = (x + sign * tab[s]) % W
            out[s, x] = reduce(src[rows, cols])
    return out


def full(img: np.ndarray, reduce=np.sum) -> np.ndarray:
    h1, h2, h3, h4 = (quadrant(img, q, reduce) for q in (1, 2, 3, 4))
    return np.concatenate([h1[::-1], h2[1:], h3[::-1][1:], h4[1:]], axis=0)


def pattern_mask(h: int, w: int, q: int, s: int, x0: int) -> np.ndarray:
    """Image pixels (inside h x w) covered by the pattern (q, s, x0)."""
    hp, wp = pow2_ceil(h), pow2_ceil(w)
    W = hp + wp
    transposed = q >= 3
    sign = 1 if q in (1, 4) else -1
    n = wp if transposed else hp
    mask = np.zeros((h, w), dtype=np.int64)
    for r in range(n):
        c = (x0 + sign * pattern_closed_form(n, s, r)) % W
        y, x = (c, r) if transposed else (r, c)
        if y < h and x < w:
            mask[y, x] += 1
    return mask
