"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: brute force along explicitly
built patterns, a textbook reduction (column sums, row sums, traces), an
invariant of the transform, or a statement of the paper.
"""
import math

import numpy as np
import pytest

import brute_force as bf

SIZES = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 5), (4, 4), (5, 3), (8, 8), (7, 12), (16, 9), (13, 32)]


def _rand(h, w, seed=0, lo=0, hi=9):
    return np.random.default_rng(seed + 31 * h + w).integers(lo, hi + 1, size=(h, w)).astype(np.float64)


# ---------------------------------------------------------------- the pattern

@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64, 256])
def test_pattern_recursion_matches_bitwise_closed_form(oracle_mod, n):
    for s in range(n):
        for y in range(n):
            assert oracle_mod.pattern_offset(n, s, y) == bf.pattern_closed_form(n, s, y)


@pytest.mark.parametrize("n", [2, 4, 8, 32, 128, 512])
def test_pattern_is_a_digital_segment(oracle_mod, n):
    """A dyadic pattern with shift s runs from column 0 at the first row to
    column s at the last (section 3.1: shift = total horizontal run over the
    h rows), moves by 0 or 1 column per row, is centrally symmetric like the
    segment it approximates, and stays within log2(n)/6 of that segment."""
    k = int(math.log2(n))
    for s in range(n):
        d = [oracle_mod.pattern_offset(n, s, y) for y in range(n)]
        assert d[0] == 0 and d[-1] == s
        assert all(b - a in (0, 1) for a, b in zip(d, d[1:]))
        assert all(d[n - 1 - y] == s - d[y] for y in range(n))
        dev = max(abs(d[y] - s * y / (n - 1)) for y in range(n))
        assert dev <= k / 6 + 1e-12
    # shift 0 is the vertical line, shift n-1 the exact 45-degree diagonal
    assert all(oracle_mod.pattern_offset(n, 0, y) == 0 for y in range(n))
    assert all(oracle_mod.pattern_offset(n, n - 1, y) == y for y in range(n))


# ------------------------------------------------------------ quadrant values

@pytest.mark.parametrize("h,w", SIZES)
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_quadrant_matches_brute_force(oracle_mod, h, w, q):
    img = _rand(h, w, seed=q)
    np.testing.assert_array_equal(oracle_mod.quadrant(img, q), bf.quadrant(img, q))


# The single-cell routines are the checker wherever the whole oracle is too
# slow (the 65536 side) and the sampled checks beside the whole-image
# comparisons, so they are pinned on their own: every (row, x0) of small
# non-square images, every quadrant, against brute force along the
# explicitly built pattern (section 2 pattern sums; section 3.3 row order).
CELL_SIZES = [(3, 5), (5, 3), (7, 12), (12, 7), (16, 9), (9, 30), (2, 13), (1, 6)]


@pytest.mark.parametrize("h,w", CELL_SIZES)
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_cell_matches_brute_force_everywhere(oracle_mod, h, w, q):
    img = _rand(h, w, seed=40 + q, lo=-7, hi=9)
    want = bf.quadrant(img, q)
    n, W = want.shape
    got = np.array([[oracle_mod.cell(img, q, s, x) for x in range(W)] for s in range(n)])
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("h,w", CELL_SIZES)
def test_full_cells_match_brute_force_everywhere(oracle_mod, h, w):
    img = _rand(h, w, seed=50, lo=-7, hi=9)
    want = bf.full(img)
    rows, W = want.shape
    rr, cc = np.meshgrid(np.arange(rows), np.arange(W), indexing="ij")
    got = oracle_mod.full_cells(img, rr.ravel(), cc.ravel()).reshape(rows, W)
    np.testing.assert_array_equal(got, want)
    # and one by one, the scalar entry point
    for r in range(rows):
        assert oracle_mod.full_cell(img, r, (3 * r + 1) % W) == want[r, (3 * r + 1) % W]


def test_full_cell_outside_the_image_is_nan(oracle_mod):
    img = _rand(5, 7)
    rows, W = oracle_mod.hough_shape(7, 5)
    assert math.isnan(oracle_mod.full_cell(img, rows, 0))
    assert math.isnan(oracle_mod.full_cell(img, -1, 0))


@pytest.mark.parametrize("h,w", [(8, 8), (5, 12), (16, 3)])
def test_full_matches_brute_force(oracle_mod, h, w):
    img = _rand(h, w, seed=7)
    np.testing.assert_array_equal(oracle_mod.full(img), bf.full(img))


@pytest.mark.parametrize("h,w", [(4, 4), (6, 10), (16, 16), (9, 30)])
def test_textbook_rows(oracle_mod, h, w):
    """Shift 0 of the vertical quadrants is the column sum, shift 0 of the
    horizontal ones the row sum; the 45-degree rows are (anti)diagonal traces
    of the periodically extended padded image."""
    img = _rand(h, w, seed=3)
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    W = hp + wp
    P = np.zeros((hp, W))
    P[:h, :w] = img
    col_sums = P.sum(axis=0)
    row_sums = np.zeros(W)
    row_sums[:h] = img.sum(axis=1)
    H = {q: oracle_mod.quadrant(img, q) for q in (1, 2, 3, 4)}
    np.testing.assert_array_equal(H[1][0], col_sums)
    np.testing.assert_array_equal(H[2][0], col_sums)
    np.testing.assert_array_equal(H[3][0], row_sums)
    np.testing.assert_array_equal(H[4][0], row_sums)
    PP = np.concatenate([P, P], axis=1)
    diag = np.array([np.trace(PP, offset=x) for x in range(W)])
    np.testing.assert_array_equal(H[1][hp - 1], diag)
    # anti-diagonals: H2[h'-1, x] = sum_y P[y, x - y]
    PPf = np.concatenate([P, P], axis=1)[:, ::-1]          # column c <- 2W-1-c
    anti = np.array([np.trace(PPf, offset=(2 * W - 1 - (x + W))) for x in range(W)])
    np.testing.assert_array_equal(H[2][hp - 1], anti)


@pytest.mark.parametrize("h,w", [(5, 7), (16, 16), (32, 9)])
def test_every_row_preserves_the_total(oracle_mod, h, w):
    """Each shift's patterns partition every row's pixels, so each Hough row
    sums to the image total."""
    img = _rand(h, w, seed=11)
    for q in (1, 2, 3, 4):
        np.testing.assert_array_equal(oracle_mod.quadrant(img, q).sum(axis=1),
                                      np.full(bf.pow2_ceil(w if q > 2 else h), img.sum()))


def test_linearity(oracle_mod):
    a, b = _rand(12, 20, 1, -5, 5), _rand(12, 20, 2, -5, 5)
    np.testing.assert_array_equal(oracle_mod.full(3 * a - 2 * b),
                                  3 * oracle_mod.full(a) - 2 * oracle_mod.full(b))


@pytest.mark.parametrize("h,w", [(8, 8), (12, 5), (3, 30), (64, 64)])
def test_junction_rows_are_shared(oracle_mod, h, w):
    """Section 3.3: consecutive quadrants are concatenated on a common edge
    row.  With the quadrant signs used here the shared rows are equal:
    column sums (q1/q2), anti-diagonals x+y (q2/q3), row sums (q3/q4)."""
    img = _rand(h, w, seed=5)
    H = {q: oracle_mod.quadrant(img, q) for q in (1, 2, 3, 4)}
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    np.testing.assert_array_equal(H[1][0], H[2][0])
    np.testing.assert_array_equal(H[2][hp - 1], H[3][wp - 1])
    np.testing.assert_array_equal(H[3][0], H[4][0])
    F = oracle_mod.full(img)
    assert F.shape == (2 * (hp + wp) - 3, hp + wp)      # section 3.3 size 2(w+h)-3


@pytest.mark.parametrize("h,w", [(8, 8), (16, 32), (32, 16)])
def test_black_zone_is_zero(oracle_mod, h, w):
    """Section 3.2 (c): patterns lying wholly in the zero extension give a
    triangle of zeros; for quadrant 1 row s that is x0 in [w', W - s)."""
    img = _rand(h, w, seed=9, lo=1, hi=9)
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    W = hp + wp
    H1 = oracle_mod.quadrant(img, 1)
    for s in range(hp):
        assert np.all(H1[s, wp:W - s] == 0)
        assert np.all(H1[s, :wp] > 0) and np.all(H1[s, W - s:] > 0)


@pytest.mark.parametrize("h,w", [(16, 16), (8, 32), (32, 8)])
def test_planted_pattern_peak(oracle_mod, h, w):
    """A binary image holding exactly one pattern gives h' (resp. w') at that
    pattern's cell, the maximum any cell can reach."""
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    for q, s, x0 in [(1, 5, 2), (2, 3, w - 1), (3, 2, h - 1), (4, 7, 0)]:
        n = hp if q <= 2 else wp
        s = min(s, n - 1)
        img = bf.pattern_mask(h, w, q, s, x0).astype(np.float64)
        assert img.sum() == n
        H = oracle_mod.quadrant(img, q)
        assert H[s, x0] == n and H.max() == n


@pytest.mark.parametrize("h,w,yp,xp", [(16, 16, 5, 9), (8, 32, 7, 20), (32, 8, 0, 0), (16, 16, 15, 15)])
def test_point_maps_to_an_angle(oracle_mod, h, w, yp, xp):
    """Sections 3.3 and 6: a single pixel gives exactly one 1 per row of the
    full image; the vertical half is one straight polyline through x0 = xp at
    the q1/q2 junction (eqs. (1) and (2)), the horizontal half another one,
    and they meet on the common row with x0 = xp + yp.  Positions stay within
    the dyadic deviation of the straight segments."""
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    W = hp + wp
    img = np.zeros((h, w))
    img[yp, xp] = 1
    F = oracle_mod.full(img)
    assert np.all(F.sum(axis=1) == 1) and np.all((F == 0) | (F == 1))
    pos = F.argmax(axis=1)
    rows = F.shape[0]
    assert pos[hp - 1] == xp                       # q1/q2 junction: vertical line through the pixel
    assert pos[2 * hp - 2] == (xp + yp) % W         # the common row of the angle
    assert pos[2 * hp + wp - 3] == yp               # q3/q4 junction: horizontal line through the pixel
    assert pos[0] == (xp - yp) % W and pos[rows - 1] == (yp - xp) % W

    def circ(a, b):
        d = (a - b) % W
        return min(d, W - d)
    dv, dh = math.log2(hp) / 6 + 1e-9, math.log2(wp) / 6 + 1e-9
    for r in range(0, 2 * hp - 1):                # first segment: x0 = xp + (r - h'+1) yp/(h'-1)
        ideal = xp + (r - (hp - 1)) * (yp / (hp - 1) if hp > 1 else 0)
        assert circ(pos[r], ideal) <= dv
    for r in range(2 * hp - 2, rows):             # second segment: from xp+yp down to yp-xp
        ideal = xp + yp - (r - (2 * hp - 2)) * (xp / (wp - 1) if wp > 1 else 0)
        assert circ(pos[r], ideal) <= dh


# ------------------------------------------------------------------- fhtshift

@pytest.mark.parametrize("h,w", [(8, 8), (16, 4), (4, 16), (1, 1), (2, 8)])
def test_fhtshift_centres_the_meaningful_zone(oracle_mod, h, w):
    """Section 5: after fhtshift every row's meaningful pixels (w + h tg a of
    them: w'+s for vertical rows, h'+s for horizontal rows) form one run
    centred in the row, black zone at both edges.  All-ones image: every
    meaningful cell is positive, every black cell zero."""
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    W = hp + wp
    img = np.zeros((hp, wp))
    img[:, :] = 1
    F = oracle_mod.full(img)
    G = oracle_mod.fhtshift_full(F, wp, hp)
    for r in range(F.shape[0]):
        q, s = oracle_mod.row_quadrant(wp, hp, r)
        run = (wp + s) if q <= 2 else (hp + s)
        nq = hp if q <= 2 else wp
        start = (nq - s) // 2
        nz = np.nonzero(G[r])[0]
        assert len(nz) == run
        assert nz[0] == start and nz[-1] == start + run - 1
        assert start + run <= W


@pytest.mark.parametrize("h,w", [(5, 7), (16, 16), (3, 40)])
def test_fhtshift_is_a_row_permutation(oracle_mod, h, w):
    img = _rand(h, w, seed=2)
    F = oracle_mod.full(img)
    G = oracle_mod.fhtshift_full(F, w, h)
    np.testing.assert_array_equal(np.sort(G, axis=1), np.sort(F, axis=1))
    np.testing.assert_array_equal(oracle_mod.fhtshift_full(G, w, h, inverse=True), F)


def test_fhtshift_matches_paper_roll_for_quadrant1(oracle_mod):
    """Section 5 gives the roll for flipped quadrant 1 as h - i/2 for row i
    (continuous); the integer roll is within half a column of it."""
    hp = wp = 64
    for i in range(hp):
        s = hp - 1 - i
        assert abs(oracle_mod.fhtshift_roll(1, hp, wp, s) - (hp - (i + 1) / 2)) <= 0.5 + 1e-12


# ---------------------------------------------------------------------- range

def test_range_params_integer_reading(oracle_mod):
    # [-15, 15] degrees at n = 1024: tan(15) * 1023 = 274.1
    assert oracle_mod.range_params(1024, -15, 15) == (275, 550)
    assert oracle_mod.range_params(1024, 0, 45) == (0, 1023)
    assert oracle_mod.range_params(64, -45, 0) == (63, 63)


@pytest.mark.parametrize("n", [2, 8, 64, 1024])
def test_range_sigma_is_a_rounded_line(oracle_mod, n):
    for S1 in (-(n - 1), -7, 0, 1, 5, n - 1):
        sig = [oracle_mod.range_sigma(n, S1, y) for y in range(n)]
        assert sig[0] == 0 and sig[-1] == S1
        assert all(abs(sig[y] - y * S1 / (n - 1)) <= 0.5 for y in range(n))
        assert all(abs(b - a) <= max(1, math.ceil(abs(S1) / (n - 1))) for a, b in zip(sig, sig[1:]))


@pytest.mark.parametrize("h,w", [(8, 8), (16, 5), (6, 20)])
def test_range_reductions(oracle_mod, h, w):
    """S1 = 0, S = n-1 is quadrant 1 itself; S1 = n-1, S = 0 shears every row
    back by y, so its single row is the anti-diagonal sum (quadrant 2's last
    row).  The transposed form reduces to quadrant 4 the same way."""
    img = _rand(h, w, seed=4)
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    np.testing.assert_array_equal(oracle_mod.range_transform(img, 0, hp - 1), oracle_mod.quadrant(img, 1))
    np.testing.assert_array_equal(oracle_mod.range_transform(img, hp - 1, 0)[0],
                                  oracle_mod.quadrant(img, 2)[hp - 1])
    np.testing.assert_array_equal(oracle_mod.range_transform(img, 0, wp - 1, transposed=True),
                                  oracle_mod.quadrant(img, 4))


@pytest.mark.parametrize("h,w,S1,S", [(8, 8, 3, 6), (16, 12, -4, 9), (16, 16, 15, 15), (4, 9, 2, 3)])
def test_range_matches_brute_force_on_sheared_image(oracle_mod, h, w, S1, S):
    """Section 4: the range transform is the quadrant-1 transform of the
    horizontally sheared image (row y rolled right by sigma(y), which adds
    S1/(n-1) to every slope), restricted to shifts 0..S.  Brute force on the
    explicitly sheared padded image."""
    img = _rand(h, w, seed=8)
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    W = hp + wp
    P = np.zeros((hp, W))
    P[:h, :w] = img
    sh = np.stack([np.roll(P[y], int(math.floor(y * S1 / (hp - 1) + 0.5))) for y in range(hp)])
    tab = bf.pattern_table(hp)
    expect = np.array([[sh[np.arange(hp), (x + tab[s]) % W].sum() for x in range(W)] for s in range(S + 1)])
    np.testing.assert_array_equal(oracle_mod.range_transform(img, S1, S), expect)


def test_range_peak_follows_planted_slope(oracle_mod):
    """A planted straight line of slope t peaks at the shift whose slope
    (s - S1)/(n-1) is closest to t, within the dyadic deviation."""
    n = 256
    S1, S = oracle_mod.range_params(n, -15, 15)
    for t in (-0.2, -0.05, 0.0, 0.1, 0.25):
        img = np.zeros((n, n))
        ys = np.arange(n)
        img[ys, np.rint(100 + t * ys).astype(int)] = 1
        R = oracle_mod.range_transform(img, S1, S)
        s_peak = np.unravel_index(R.argmax(), R.shape)[0]
        assert abs((s_peak - S1) - t * (n - 1)) <= 3


@pytest.mark.parametrize("h,w", [(32, 32), (16, 40), (64, 24)])
def test_range_sheared_black_zone_moves_without_cyclic_effect(oracle_mod, h, w):
    """Section 4, Fig. 5: after a horizontal shear by arctg(1/2) the zero
    extension keeps the sheared image from wrapping around, and the black
    zone only moves and changes its shape.

    Built independently of the oracle's recurrence: with
    f_s(y) = D(s, y) - sigma(y) (pattern offset minus the row's shear, both
    moving by 0 or 1 column per row, so f_s takes every value between its
    extremes), the pattern of row s at x0 meets the image iff
    x0 + f_s(y) is in [0, w) for some image row y.  On an all-white image
    the zero cells of row s are therefore exactly one cyclic run of
    W - w - (max f_s - min f_s) columns starting at w - min f_s.  And on a white cross the
    cyclic shear equals the explicit shear of the image onto a wider canvas
    (no pixel wraps round)."""
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    W = hp + wp
    n = hp
    S1 = (n - 1) // 2                      # shear of about arctg(1/2): sigma(y) ~ y / 2
    sigma = [math.floor((2 * y * S1 + (n - 1)) / (2 * (n - 1))) for y in range(n)]
    # all-white image: the zero cells of every row form the predicted run
    R = oracle_mod.range_transform(np.ones((h, w)), S1, n - 1)
    for s in range(n):
        f = [bf.pattern_closed_form(n, s, y) - sigma[y] for y in range(h)]
        lo, hi = min(f), max(f)
        zero = np.zeros(W, dtype=bool)
        assert W - w - (hi - lo) > 0        # the run never closes: no cyclic effect
        for k in range(W - w - (hi - lo)):
            zero[(w - lo + k) % W] = True
        assert np.array_equal(R[s] == 0, zero), s
        assert np.all(R[s][~zero] > 0)
    # a white cross: the cyclic shear equals the explicit one on a canvas wide
    # enough that nothing can wrap, summed along the patterns by brute force
    cross = np.zeros((h, w))
    cross[h // 2 - 1:h // 2 + 1, :] = 1.0
    cross[:, w // 2 - 1:w // 2 + 1] = 1.0
    canvas = np.zeros((n, W))
    for y in range(h):
        canvas[y, sigma[y]:sigma[y] + w] = cross[y]       # sigma(y) + w <= W: no wrap
    assert max(sigma) + w <= W
    tab = bf.pattern_table(n)
    want = np.array([[canvas[np.arange(n), (x + tab[s]) % W].sum() for x in range(W)] for s in range(n)])
    np.testing.assert_array_equal(oracle_mod.range_transform(cross, S1, n - 1), want)


# -------------------------------------------------------------------- adjoint

@pytest.mark.parametrize("h,w", [(1, 1), (3, 5), (8, 8), (16, 7), (5, 33)])
def test_adjoint_inner_product_identity(oracle_mod, h, w):
    """<F x, y> = <x, F^T y> exactly on integers."""
    x = _rand(h, w, seed=1, lo=-50, hi=50)
    rows, W = oracle_mod.hough_shape(w, h)
    y = np.random.default_rng(5).integers(-50, 51, size=(rows, W)).astype(np.float64)
    lhs = float(np.sum(oracle_mod.full(x) * y))
    rhs = float(np.sum(x * oracle_mod.adjoint_full(y, w, h)))
    assert lhs == rhs
    for q in (1, 2, 3, 4):
        n = bf.pow2_ceil(h) if q <= 2 else bf.pow2_ceil(w)
        yq = y[:n]
        assert float(np.sum(oracle_mod.quadrant(x, q) * yq)) == \
            float(np.sum(x * oracle_mod.adjoint_quadrant(yq, w, h, q)))


@pytest.mark.parametrize("h,w", [(8, 8), (6, 11)])
def test_adjoint_of_an_impulse_is_its_pattern(oracle_mod, h, w):
    """Back-projecting one Hough cell marks exactly that pattern's pixels."""
    hp, wp = bf.pow2_ceil(h), bf.pow2_ceil(w)
    W = hp + wp
    for q, s, x0 in [(1, 3, 1), (2, hp - 1, 4), (3, 2, 0), (4, wp - 1, W - 2)]:
        n = hp if q <= 2 else wp
        g = np.zeros((n, W))
        g[s, x0] = 1
        np.testing.assert_array_equal(oracle_mod.adjoint_quadrant(g, w, h, q),
                                      bf.pattern_mask(h, w, q, s, x0))


# ------------------------------------------------------- single precision mode

def test_single_mode_rounds_each_add(oracle_mod):
    """The binary32 mode evaluates the same add tree in float: results equal a
    numpy float32 stage-by-stage evaluation on a case where float rounding
    differs from double."""
    rng = np.random.default_rng(0)
    img = (rng.standard_normal((16, 16)) * np.float32(1e4)).astype(np.float32)
    img[0, 0] = np.float32(1e8)
    h1_32 = oracle_mod.quadrant(img, 1, single=True)
    # float32 stage recurrence, written with numpy roll on whole rows
    n, W = 16, 32
    A = np.zeros((n, W), dtype=np.float32)
    A[:, :16] = img
    blk = 1
    while blk < n:
        B = np.empty_like(A)
        for row in range(n):
            base = row - row % (2 * blk)
            t = row - base
            B[row] = A[base + (t >> 1)] + np.roll(A[base + blk + (t >> 1)], -(t - (t >> 1)))
        A, blk = B, blk * 2
    np.testing.assert_array_equal(h1_32, A.astype(np.float64))
    assert not np.array_equal(h1_32, oracle_mod.quadrant(img, 1))


# ------------------------------------------------- integer facts of the paper

def test_paper_structure_fixture(oracle_mod):
    """Sizes and row boundaries stated in sections 3.1, 3.3 and 5
    (tests/golden/paper_structure.json), on pow2 sides where h' = h."""
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_structure.json")))
    for ex in fx["examples"]:
        w, h = ex["w"], ex["h"]
        env = {"w": w, "h": h}
        img = np.ones((h, w))
        assert oracle_mod.quadrant(img, 1).shape == (eval(fx["quadrant_result_size"]["rows"], env),
                                                     eval(fx["quadrant_result_size"]["cols"], env))
        rows = eval(fx["full_image_rows"]["rows"], env)
        assert oracle_mod.full(img).shape[0] == rows
        b = fx["row_to_quadrant_boundaries"]
        q1e, q2e, q3e = (eval(b[k], env) for k in ("q1_end", "q2_end", "q3_end"))
        for r in range(rows):
            q, _ = oracle_mod.row_quadrant(w, h, r)
            assert q == (1 if r < q1e else 2 if r < q2e else 3 if r < q3e else 4)
        # roll of flipped quadrant 1: row 0 (shift h-1) by ~h, last row (shift 0) by h/2
        assert abs(oracle_mod.fhtshift_roll(1, h, w, h - 1) - eval(fx["fhtshift_q1_roll"]["row0"], env)) <= 1
        assert oracle_mod.fhtshift_roll(1, h, w, 0) == eval(fx["fhtshift_q1_roll"]["last_row"], env)


# ---- the max transform (section 1: the transform generalises to any
# associative, commutative operation along the same patterns)

@pytest.mark.parametrize("h,w", [(1, 1), (3, 5), (8, 8), (7, 12), (16, 9)])
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_max_quadrant_matches_brute_force(oracle_mod, h, w, q):
    img = _rand(h, w, seed=40 + q, lo=-5, hi=20)
    np.testing.assert_array_equal(oracle_mod.quadrant_op(img, q, "max"), bf.quadrant(img, q, np.max))


@pytest.mark.parametrize("h,w", [(8, 8), (5, 12), (16, 3)])
def test_max_full_matches_brute_force(oracle_mod, h, w):
    img = _rand(h, w, seed=9, lo=0, hi=30)
    np.testing.assert_array_equal(oracle_mod.full_op(img, "max"), bf.full(img, np.max))


def test_max_textbook_rows(oracle_mod):
    """Shift 0 of the vertical quadrants is the column maximum of the padded
    image; of the horizontal quadrants, the row maximum."""
    img = _rand(12, 7, seed=3, lo=1, hi=50)
    hp, wp = 16, 8
    P = np.zeros((hp, hp + wp))
    P[:12, :7] = img
    np.testing.assert_array_equal(oracle_mod.quadrant_op(img, 1, "max")[0], P.max(axis=0))
    Pt = np.zeros((wp, hp + wp))
    Pt[:7, :12] = img.T
    np.testing.assert_array_equal(oracle_mod.quadrant_op(img, 4, "max")[0], Pt.max(axis=0))


def test_max_row_maximum_is_the_image_maximum(oracle_mod):
    """For every shift the patterns x0 = 0..W-1 partition the padded image,
    so the maximum over any Hough row is the maximum over the padded image."""
    img = _rand(9, 13, seed=5, lo=-7, hi=7)
    gmax = max(img.max(), 0.0)  # the zero padding takes part
    for q in (1, 2, 3, 4):
        H = oracle_mod.quadrant_op(img, q, "max")
        np.testing.assert_array_equal(H.max(axis=1), np.full(H.shape[0], gmax))


def test_max_of_binary_image_is_or(oracle_mod):
    """On a 0/1 image max is the logical OR: a cell is 1 exactly when its
    pattern's sum is positive."""
    img = (np.random.default_rng(11).random((16, 16)) < 0.1).astype(np.float64)
    np.testing.assert_array_equal(oracle_mod.full_op(img, "max"), (oracle_mod.full(img) > 0).astype(np.float64))


# ---- adjoint of the angle-range transform (section 4)

RANGE_CASES = [(8, 8, 0, 7, False), (8, 8, 3, 6, False), (16, 12, -5, 9, False), (13, 16, 7, 15, False),
               (16, 16, -15, 15, False), (12, 7, 2, 5, True), (9, 16, -3, 4, True), (8, 16, 0, 15, True)]


@pytest.mark.parametrize("h,w,S1,S,tr", RANGE_CASES)
def test_range_adjoint_inner_product_identity(oracle_mod, h, w, S1, S, tr):
    """<R x, g> = <x, R^T g> exactly on integers, R the (brute-force pinned)
    range transform."""
    rng = np.random.default_rng(h * 31 + w + S1)
    x = rng.integers(-50, 51, size=(h, w)).astype(np.float64)
    Rx = oracle_mod.range_transform(x, S1, S, tr)
    g = rng.integers(-50, 51, size=Rx.shape).astype(np.float64)
    lhs = int(np.sum(Rx.astype(np.int64) * g.astype(np.int64)))
    rhs = int(np.sum(x.astype(np.int64) * oracle_mod.range_adjoint(g, w, h, S1, S, tr).astype(np.int64)))
    assert lhs == rhs


def test_range_adjoint_unsheared_full_range_is_the_quadrant_adjoint(oracle_mod):
    """S1 = 0, S = n - 1: the range is quadrant 1 (4 when transposed), so its
    adjoint is the quadrant adjoint."""
    rng = np.random.default_rng(2)
    h, w = 16, 11
    g1 = rng.integers(-9, 10, size=(16, 32)).astype(np.float64)
    np.testing.assert_array_equal(oracle_mod.range_adjoint(g1, w, h, 0, 15, False),
                                  oracle_mod.adjoint_quadrant(g1, w, h, 1))
    g4 = rng.integers(-9, 10, size=(16, 32)).astype(np.float64)
    np.testing.assert_array_equal(oracle_mod.range_adjoint(g4, w, h, 0, 15, True),
                                  oracle_mod.adjoint_quadrant(g4, w, h, 4))


# ---- scale along the sheared axis in the first iteration (section 4);
# the nearest-sample resampling is a reading of that section (the paper fixes none)

@pytest.mark.parametrize("tr", [False, True])
def test_scale_one_is_the_plain_range(oracle_mod, tr):
    img = _rand(12, 9, seed=1)
    np.testing.assert_array_equal(oracle_mod.range_scaled(img, 3, 3, 2, 5, tr), oracle_mod.range_transform(img, 2, 5, tr))


def test_scale_two_duplicates_columns(oracle_mod):
    img = _rand(10, 7, seed=2)
    np.testing.assert_array_equal(oracle_mod.range_scaled(img, 2, 1, 3, 6),
                                  oracle_mod.range_transform(np.repeat(img, 2, axis=1), 3, 6))


def test_scale_half_keeps_every_other_column(oracle_mod):
    img = _rand(10, 16, seed=3)
    np.testing.assert_array_equal(oracle_mod.range_scaled(img, 1, 2, -2, 7),
                                  oracle_mod.range_transform(img[:, ::2], -2, 7))


def test_scale_transposed_scales_rows(oracle_mod):
    img = _rand(6, 11, seed=4)
    np.testing.assert_array_equal(oracle_mod.range_scaled(img, 3, 1, 1, 7, True),
                                  oracle_mod.range_transform(np.repeat(img, 3, axis=0), 1, 7, True))


def test_scale_maps_inclination_by_the_tangent(oracle_mod):
    """A line of slope t = tan(beta) peaks, after scaling by alpha, at the
    shift of slope alpha * t (section 4: beta' = arctg(alpha tg beta)),
    to within the dyadic deviation."""
    n = 256
    for alpha_num, alpha_den, t in [(2, 1, 0.3), (2, 1, 0.45), (3, 2, 0.5), (1, 2, 0.9)]:
        img = np.zeros((n, n))
        ys = np.arange(n)
        img[ys, np.rint(20 + t * ys).astype(int)] = 1.0
        R = oracle_mod.range_scaled(img, alpha_num, alpha_den, 0, n - 1)
        s_peak = int(np.unravel_index(np.argmax(R), R.shape)[0])
        assert abs(s_peak - (alpha_num / alpha_den) * t * (n - 1)) <= 4.0, (alpha_num, alpha_den, t, s_peak)
