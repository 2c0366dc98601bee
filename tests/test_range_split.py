"""Splitting an inclination range into angle-range calls (section 4): host
logic, no GPU.  Every integer slope step of the requested range is covered,
in the right family, by a call with valid (S1, S)."""
import math

import pytest

from paper_1811_06378_amd import fht


def _steps(n, lo, hi):
    return set(range(math.floor((n - 1) * math.tan(math.radians(lo)) + 1e-9),
                     math.ceil((n - 1) * math.tan(math.radians(hi)) - 1e-9) + 1))


@pytest.mark.parametrize("h,w", [(64, 64), (100, 37), (1024, 1024), (5, 300)])
@pytest.mark.parametrize("lo,hi", [(-15, 15), (-45, 45), (-90, 90), (30, 80), (-80, -50), (0, 0), (44, 46),
                                   (-60, 10), (89, 90)])
def test_pieces_cover_the_range(h, w, lo, hi):
    pieces = fht.range_pieces(h, w, lo, hi)
    hp = 1 << max(0, (h - 1).bit_length())
    wp = 1 << max(0, (w - 1).bit_length())
    vert, horiz = set(), set()
    for p in pieces:
        n = p["n"]
        assert n == (wp if p["transposed"] else hp)
        assert 0 <= p["S"] <= n - 1 and -(n - 1) <= p["S1"] <= n - 1
        k0, k1 = p["k"]
        assert p["S1"] == -k0 and p["S"] == k1 - k0
        (horiz if p["transposed"] else vert).update(range(k0, k1 + 1))
    want_v = _steps(hp, max(lo, -45), min(hi, 45)) if hi >= -45 and lo <= 45 else set()
    want_h = set()
    if hi > 45:
        want_h |= _steps(wp, 90 - hi, 90 - max(lo, 45))
    if lo < -45:
        want_h |= _steps(wp, -90 - min(hi, -45), -90 - lo)
    assert vert == want_v
    assert horiz == want_h


def test_pieces_reject_bad_ranges():
    with pytest.raises(ValueError):
        fht.range_pieces(64, 64, 10, -10)
    with pytest.raises(ValueError):
        fht.range_pieces(64, 64, -100, 0)


def test_one_call_per_narrow_range():
    # [-15, 15] at 1024 is one call, the integer reading of the bench workload
    (p,) = fht.range_pieces(1024, 1024, -15, 15)
    assert (p["S1"], p["S"], p["transposed"]) == (275, 550, False)
