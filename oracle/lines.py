"""From Hough cells back to image lines, written from the definitions
(sections 3.2 and 3.3).  TEST INFRASTRUCTURE ONLY: like the rest of this
package it is imported by the tests, never by the library.

  cell_segment(w, h, quads, row, x0, shifted)
      The cell's dyadic pattern, walked row by row on the padded source with
      cyclic columns (section 3.2, cases a and b), cut to the pixels inside
      the h x w image: the first and last of them and their number, or None
      when the pattern runs in the zero extension only (case c, the black
      zone).  A full-image row is attributed to its quadrant and local shift
      by the row order of section 3.3; an fhtshift-ed cell is rolled back
      first (section 5).
  local_maxima(H, radius, threshold)
      Every cell above the threshold that beats each other cell of its
      (2 radius + 1)^2 neighbourhood: strictly larger, or equal with a larger
      linear index (so a plateau yields one cell).  Columns are cyclic (x0
      is taken mod W), rows are clipped.
  strongest_maxima(H, radius, threshold, k)
      The k largest of those, by the same definition, for images too large
      to scan every neighbourhood in Python.
"""
from __future__ import annotations

import numpy as np

from . import oracle as _o


def _quadrant_and_shift(w, h, quads, row):
    hp, wp = _o.next_pow2(h), _o.next_pow2(w)
    if quads == "full":
        q, s = _o.row_quadrant(w, h, row)
        if q == 0:
            raise ValueError("row %d outside the full Hough image" % row)
        return q, s
    q = int(quads)
    n = hp if q <= 2 else wp
    if not 0 <= row < n:
        raise ValueError("row %d outside quadrant %d" % (row, q))
    return q, row


def cell_segment(w: int, h: int, row: int, x0: int, quads="full", shifted: bool = False):
    """((xa, ya), (xb, yb), pixels) of Hough cell (row, x0), or None."""
    hp, wp = _o.next_pow2(h), _o.next_pow2(w)
    W = hp + wp
    if not 0 <= x0 < W:
        raise ValueError("x0 %d outside 0..%d" % (x0, W - 1))
    q, s = _quadrant_and_shift(w, h, quads, row)
    n = hp if q <= 2 else wp
    if shifted:
        if quads != "full":
            raise ValueError("fhtshift applies to the full Hough image only")
        x0 = (x0 - _o.fhtshift_roll(q, hp, wp, s)) % W
    direction = 1 if q in (1, 4) else -1
    pixels = []
    for r in range(n):
        c = (x0 + direction * _o.pattern_offset(n, s, r)) % W
        x, y = (r, c) if q >= 3 else (c, r)
        if x < w and y < h:
            pixels.append((x, y))
    if not pixels:
        return None
    return pixels[0], pixels[-1], len(pixels)


def _beats_neighbours(H, r, c, radius):
    rows, cols = H.shape
    v = H[r, c]
    me = r * cols + c
    for rr in range(max(0, r - radius), min(rows, r + radius + 1)):
        for dc in range(-radius, radius + 1):
            cc = (c + dc) % cols
            if rr == r and cc == c:
                continue
            u = H[rr, cc]
            if u > v or (u == v and rr * cols + cc < me):
                return False
    return True


def local_maxima(H, radius: int, threshold: float):
    """[(value, row, col)] by decreasing value, ties by index."""
    H = np.asarray(H)
    rows, cols = H.shape
    if 2 * radius + 1 > cols:
        raise ValueError("the neighbourhood must fit in one row")
    out = []
    for r, c in zip(*np.nonzero(H > threshold)):
        if _beats_neighbours(H, int(r), int(c), radius):
            out.append((H[r, c].item(), int(r), int(c)))
    return sorted(out, key=lambda e: (-e[0], e[1], e[2]))


def strongest_maxima(H, radius: int, threshold: float, k: int):
    """The first k entries of local_maxima(H, radius, threshold).

    A cell that beats every neighbour equals the maximum of its
    neighbourhood, so the candidates are the cells equal to a maximum filter
    of the image (cyclic columns, clipped rows); they are confirmed one by
    one, largest first, with the exact rule."""
    from scipy import ndimage

    H = np.asarray(H)
    rows, cols = H.shape
    size = 2 * radius + 1
    lowest = -np.inf if H.dtype.kind == "f" else np.iinfo(H.dtype).min
    M = ndimage.maximum_filter(H, size=(size, size), mode=("constant", "wrap"), cval=lowest)
    cand = np.nonzero((H == M) & (H > threshold))
    vals = H[cand]
    order = np.lexsort((cand[1], cand[0], -vals.astype(np.float64)))
    out = []
    for i in order:
        r, c = int(cand[0][i]), int(cand[1][i])
        if _beats_neighbours(H, r, c, radius):
            out.append((H[r, c].item(), r, c))
            if len(out) == k:
                break
    return out
