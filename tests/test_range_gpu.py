"""Angle-range adjoint and split ranges on the GPU (section 4).

Range adjoint: int32 bit-exact against the oracle's transpose and the exact
inner-product identity; float32 bit-exact against the oracle's binary32
mode and within 1e-5 of the float64 transpose of |g|.  range_any: every
piece equals the oracle's range transform of that piece."""
import numpy as np
import pytest
import torch

import oracle
import gpu_util as P
from gpu_util import assert_close_fp, assert_equal, dev, host
from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu

# (h, w, S1, S, transposed): tiny (direct kernel), one and two passes, ragged,
# negative S1, transposed
CASES = [(4, 4, 1, 2, False), (2, 5, 1, 1, False), (8, 8, 0, 7, False), (16, 20, -5, 10, False),
         (64, 64, 20, 40, False), (100, 70, -30, 100, False), (256, 256, 68, 136, False),
         (300, 520, 40, 200, True), (520, 300, -100, 300, False), (1024, 1024, 275, 550, False),
         (37, 130, 60, 90, True)]


def _grad(shape, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "i32":
        return rng.integers(-1000, 1001, size=shape).astype(np.int32)
    return rng.standard_normal(shape).astype(np.float32)


@pytest.mark.parametrize("h,w,S1,S,tr", CASES)
def test_range_adjoint_int_exact(h, w, S1, S, tr):
    rows, cols = fht.range_shape(w, h, S1, S, tr)
    g = _grad((rows, cols), "i32", seed=h + w + S)
    got = host(P.range_adjoint(dev(g), w, h, S1, S, tr))
    want = oracle.range_adjoint(g.astype(np.float64), w, h, S1, S, tr)
    assert_equal(got.astype(np.float64), want, "range adjoint %dx%d S1=%d S=%d tr=%d" % (h, w, S1, S, tr))


@pytest.mark.parametrize("h,w,S1,S,tr", CASES)
def test_range_adjoint_float(h, w, S1, S, tr):
    rows, cols = fht.range_shape(w, h, S1, S, tr)
    g = _grad((rows, cols), "f32", seed=7 * h + w)
    got = host(P.range_adjoint(dev(g), w, h, S1, S, tr))
    g64 = g.astype(np.float64)
    assert_equal(got.astype(np.float64), oracle.range_adjoint(g64, w, h, S1, S, tr, single=True),
                 "range adjoint f32 vs binary32 oracle")
    assert_close_fp(got, oracle.range_adjoint(g64, w, h, S1, S, tr),
                    oracle.range_adjoint(np.abs(g64), w, h, S1, S, tr), "range adjoint f32 vs float64")


@pytest.mark.parametrize("h,w,S1,S,tr", [(64, 64, 20, 40, False), (300, 520, 40, 200, True),
                                         (1024, 1024, 275, 550, False)])
def test_range_inner_product_identity_on_gpu(h, w, S1, S, tr):
    """<R x, g> = <x, R^T g> with both sides from the GPU, in int64."""
    rng = np.random.default_rng(3)
    x = rng.integers(-100, 101, size=(h, w)).astype(np.int32)
    Rx = host(P.range_transform(dev(x), S1, S, tr)).astype(np.int64)
    g = rng.integers(-100, 101, size=Rx.shape).astype(np.int32)
    Rtg = host(P.range_adjoint(dev(g), w, h, S1, S, tr)).astype(np.int64)
    assert int(np.sum(Rx * g)) == int(np.sum(x.astype(np.int64) * Rtg))


def test_range_autograd_weighted_loss():
    """loss = sum(Wt * R(x)^2): the gradient is 2 R^T(Wt * R(x)), checked
    against the float64 oracle composition."""
    h = w = 128
    S1, S = fht.range_params(128, -20, 25)
    x = synth.random_image(h, w, "f32", seed=12)
    Wt = np.random.default_rng(5).random(fht.range_shape(w, h, S1, S)).astype(np.float32)
    xt = dev(x).requires_grad_(True)
    y = fht.RangeFunction.apply(xt, S1, S, False)
    (dev(Wt) * y * y).sum().backward()
    got = host(xt.grad)
    R = oracle.range_transform(x.astype(np.float64), S1, S)
    want = 2.0 * oracle.range_adjoint(Wt.astype(np.float64) * R, w, h, S1, S)
    bound = 2.0 * oracle.range_adjoint(np.abs(Wt.astype(np.float64) * R), w, h, S1, S)
    assert np.all(np.abs(got - want) <= 1e-4 * bound + 1e-6)


@pytest.mark.parametrize("h,w,lo,hi", [(64, 64, -90, 90), (100, 37, 30, 80), (37, 100, -80, -50),
                                       (256, 256, -45, 45), (300, 200, -60, 10)])
def test_range_any_pieces(h, w, lo, hi):
    img = synth.random_image(h, w, "u8", seed=2)
    outs = fht.range_any(dev(img), lo, hi)
    assert len(outs) >= 1
    for p, H in outs:
        want = oracle.range_transform(img.astype(np.float64), p["S1"], p["S"], transposed=p["transposed"])
        assert_equal(host(H).astype(np.float64), want, "range_any piece %s" % (p,))


# scaled range (section 4 scale in the first iteration; nearest-sample reading)
SCALED = [(64, 64, 2, 1, 0, 63, False), (64, 64, 1, 2, 5, 40, False), (100, 70, 3, 2, -10, 90, False),
          (33, 130, 2, 3, 20, 60, False), (37, 50, 5, 1, 0, 63, True), (120, 90, 1, 3, -7, 20, True),
          (256, 256, 2, 1, 0, 255, False), (4, 4, 2, 1, 1, 3, False), (3, 9, 1, 2, 0, 3, False)]


@pytest.mark.parametrize("h,w,num,den,S1,S,tr", SCALED)
@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_range_scaled(h, w, num, den, S1, S, tr, kind):
    img = synth.random_image(h, w, kind, seed=30 + num)
    got = host(P.range_scaled(dev(img), num, den, S1, S, tr))
    want = oracle.range_scaled(img.astype(np.float64), num, den, S1, S, tr, single=(kind == "f32"))
    assert_equal(got.astype(np.float64), want, "range scaled %dx%d %d/%d S1=%d S=%d tr=%d" % (h, w, num, den, S1, S, tr))
