"""Pins of the oracle's way back from Hough cells to image lines
(sections 3.2, 3.3, 5): the cell -> segment walk against the pattern's
pixels built independently (tests/brute_force.py), and the local-maximum
rule on configurations whose answer is fixed by hand."""
import numpy as np
import pytest

import brute_force as bf
import oracle
from oracle import lines


def _expected(h, w, q, s, x0):
    mask = bf.pattern_mask(h, w, q, s, x0)
    ys, xs = np.nonzero(mask)
    if len(ys) == 0:
        return None
    order = np.argsort(xs if q >= 3 else ys, kind="stable")
    ys, xs = ys[order], xs[order]
    return (int(xs[0]), int(ys[0])), (int(xs[-1]), int(ys[-1])), int(mask.sum())


@pytest.mark.parametrize("h,w", [(1, 1), (4, 4), (5, 7), (8, 8), (16, 12), (13, 32), (30, 9)])
def test_segment_of_every_full_cell_is_its_pattern(h, w):
    rows, W = oracle.hough_shape(w, h)
    for r in range(rows):
        q, s = oracle.row_quadrant(w, h, r)
        for x0 in range(W):
            assert lines.cell_segment(w, h, r, x0) == _expected(h, w, q, s, x0), (r, x0)


@pytest.mark.parametrize("h,w", [(8, 8), (16, 12), (13, 32)])
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_segment_of_single_quadrant_rows(h, w, q):
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    n = hp if q <= 2 else wp
    for s in range(n):
        for x0 in range(hp + wp):
            assert lines.cell_segment(w, h, s, x0, quads=q) == _expected(h, w, q, s, x0)


@pytest.mark.parametrize("h,w", [(8, 8), (16, 12)])
def test_shifted_cell_is_the_rolled_cell(h, w):
    """fhtshift rolls row r right by its roll (section 5): the shifted cell at
    x0 + roll is the unshifted cell x0 (roll taken from the fhtshift of an
    impulse image by the oracle, not from the segment code)."""
    rows, W = oracle.hough_shape(w, h)
    for r in range(rows):
        imp = np.zeros((rows, W))
        imp[r, 3] = 1.0
        roll = (int(np.argmax(oracle.fhtshift_full(imp, w, h)[r])) - 3) % W
        for x0 in range(W):
            assert lines.cell_segment(w, h, r, (x0 + roll) % W, shifted=True) == lines.cell_segment(w, h, r, x0)


def test_black_zone_and_step_one():
    """Section 3.2: quadrant 1 cells x0 in [w', W - s) see only the zero
    extension (case c); a cell with x0 + s inside the image runs from (x0, 0)
    to (x0 + s, h - 1) (step 1)."""
    h = w = 16
    for s in range(16):
        for x0 in range(16, 32 - s):
            assert lines.cell_segment(w, h, s, x0, quads=1) is None
        for x0 in range(0, 16 - s):
            assert lines.cell_segment(w, h, s, x0, quads=1) == ((x0, 0), (x0 + s, h - 1), h)


def test_maxima_single_spike_and_threshold():
    H = np.zeros((9, 12), dtype=np.int32)
    H[4, 7] = 5
    assert lines.local_maxima(H, 2, 0) == [(5, 4, 7)]
    assert lines.local_maxima(H, 2, 5) == []          # strictly above the threshold


def test_maxima_plateau_keeps_the_smallest_index():
    H = np.zeros((6, 10), dtype=np.float32)
    H[2:4, 3:6] = 2.0
    assert lines.local_maxima(H, 1, 0.5) == [(2.0, 2, 3)]


def test_maxima_suppression_within_the_radius_only():
    H = np.zeros((10, 20), dtype=np.int32)
    H[5, 5], H[5, 8], H[5, 14] = 9, 7, 3
    assert lines.local_maxima(H, 3, 0) == [(9, 5, 5), (3, 5, 14)]
    assert lines.local_maxima(H, 2, 0) == [(9, 5, 5), (7, 5, 8), (3, 5, 14)]


def test_maxima_columns_wrap_rows_do_not():
    H = np.zeros((8, 16), dtype=np.int32)
    H[3, 0], H[3, 15] = 9, 4        # neighbours across the cyclic column edge
    H[0, 8], H[7, 8] = 6, 5         # first and last row are not neighbours
    assert lines.local_maxima(H, 2, 0) == [(9, 3, 0), (6, 0, 8), (5, 7, 8)]


@pytest.mark.parametrize("seed", range(4))
def test_strongest_maxima_is_the_head_of_local_maxima(seed):
    rng = np.random.default_rng(seed)
    H = rng.integers(0, 12, size=(40, 57)).astype(np.int32)     # many ties
    for radius in (1, 2, 4):
        full = lines.local_maxima(H, radius, 2)
        assert lines.strongest_maxima(H, radius, 2, 10) == full[:10]
    F = rng.random((33, 64)).astype(np.float32)
    assert lines.strongest_maxima(F, 3, 0.1, 25) == lines.local_maxima(F, 3, 0.1)[:25]
