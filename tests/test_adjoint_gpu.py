"""Adjoint parity on the GPU: F^T through the C ABI vs the oracle's transpose,
the exact inner-product identity on integers, and autograd."""
import numpy as np
import pytest
import torch

import oracle
import gpu_util as P
from gpu_util import assert_close_fp, assert_equal, dev, host
from paper_1811_06378_amd import fht
from paper_1811_06378_amd import synth

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (2, 3), (4, 4), (5, 13), (8, 8), (16, 16), (9, 40), (64, 64), (33, 100), (129, 257),
         (300, 520), (520, 300)]


def _grad(h, w, kind, seed=0, quads="full"):
    rows, cols = fht.hough_shape(w, h, quads)
    rng = synth.rng_for("adjoint-grad", seed, h * 7919 + w)
    if kind == "i32":
        return rng.integers(-100, 101, size=(rows, cols), dtype=np.int32)
    return rng.standard_normal((rows, cols), dtype=np.float32)


@pytest.mark.parametrize("h,w", SIZES)
def test_adjoint_int_exact(h, w):
    g = _grad(h, w, "i32")
    got = host(P.adjoint(dev(g), w, h))
    assert_equal(got.astype(np.float64), oracle.adjoint_full(g.astype(np.float64), w, h), "adjoint i32")


@pytest.mark.parametrize("h,w", SIZES)
def test_adjoint_float(h, w):
    g = _grad(h, w, "f32", seed=1)
    got = host(P.adjoint(dev(g), w, h))
    assert_equal(got.astype(np.float64), oracle.adjoint_full(g, w, h, single=True), "adjoint f32 vs binary32")
    assert_close_fp(got, oracle.adjoint_full(g, w, h), oracle.adjoint_full(np.abs(g), w, h), "adjoint f32")


# image passes run in quadrant order, as mirror pairs (1 and 2, 3 and 4) or
# single quadrants, the later ones adding to the stored gradient: every mix
SUBSETS = [[1], [2], [3], [4], [2, 4], [1, 2], [3, 4], [2, 3], [1, 2, 3], [1, 2, 4], [1, 3, 4], [2, 3, 4]]


@pytest.mark.parametrize("h,w", [(8, 8), (16, 24), (33, 100), (300, 520)])
@pytest.mark.parametrize("quads", SUBSETS)
def test_adjoint_quadrant_subsets(h, w, quads):
    g = _grad(h, w, "i32", seed=2, quads=quads)
    got = host(P.adjoint(dev(g), w, h, quads=quads))
    hp, wp = oracle.next_pow2(h), oracle.next_pow2(w)
    want = np.zeros((h, w))
    r = 0
    for q in sorted(quads):
        n = hp if q <= 2 else wp
        want = want + oracle.adjoint_quadrant(g[r:r + n].astype(np.float64), w, h, q)
        r += n
    assert_equal(got.astype(np.float64), want, "adjoint quads %s" % quads)


@pytest.mark.parametrize("h,w", [(3, 40), (40, 3), (16, 24), (100, 33), (300, 520)])
@pytest.mark.parametrize("quads", SUBSETS)
def test_adjoint_quadrant_subsets_float_order(h, w, quads):
    """float32 subsets bit for bit: each quadrant's binary32 transpose, summed
    in binary32 in quadrant order."""
    g = _grad(h, w, "f32", seed=6, quads=quads)
    got = host(P.adjoint(dev(g), w, h, quads=quads))
    hp, wp = oracle.next_pow2(h), oracle.next_pow2(w)
    want = None
    r = 0
    for q in sorted(quads):
        n = hp if q <= 2 else wp
        c = oracle.adjoint_quadrant(g[r:r + n], w, h, q, single=True).astype(np.float32)
        want = c if want is None else (want + c).astype(np.float32)
        r += n
    assert_equal(got.astype(np.float64), want.astype(np.float64), "adjoint f32 quads %s" % quads)


@pytest.mark.parametrize("h,w", [(8, 8), (13, 5), (300, 520)])
def test_adjoint_shifted(h, w):
    g = _grad(h, w, "i32", seed=3)
    got = host(P.adjoint(dev(g), w, h, shifted=True))
    unshift = oracle.fhtshift_full(g.astype(np.float64), w, h, inverse=True)
    assert_equal(got.astype(np.float64), oracle.adjoint_full(unshift, w, h), "adjoint shifted")


@pytest.mark.parametrize("h,w", [(64, 64), (300, 520), (1024, 1024)])
def test_inner_product_identity_int32(h, w):
    """<F x, y> = <x, F^T y> exactly, both sides from the GPU kernels."""
    x = synth.int_image(h, w, seed=4)
    y = _grad(h, w, "i32", seed=5)
    Fx = host(P.forward(dev(x))).astype(np.int64)
    Fty = host(P.adjoint(dev(y), w, h)).astype(np.int64)
    assert int(np.sum(Fx * y.astype(np.int64))) == int(np.sum(x.astype(np.int64) * Fty))


def test_autograd_matches_adjoint_and_fd():
    """loss = sum(Wt * H^2): backward through FHTFunction equals 2 F^T(Wt*H),
    and a float64 central difference along a random direction agrees."""
    h, w = 32, 48
    x = synth.normal1024(0, batch=1, size=64)[0][:h, :w].copy()
    rows, cols = fht.hough_shape(w, h)
    Wt = synth.weight_map((rows, cols), 0)
    xt = dev(x).requires_grad_(True)
    H = fht.FHTFunction.apply(xt)
    loss = (dev(Wt) * H * H).sum()
    loss.backward()
    g = host(xt.grad).astype(np.float64)
    F64 = oracle.full(x.astype(np.float64))
    g64 = oracle.adjoint_full(2.0 * Wt.astype(np.float64) * F64, w, h)
    scale = oracle.adjoint_full(2.0 * Wt.astype(np.float64) * oracle.full(np.abs(x).astype(np.float64)), w, h)
    assert np.all(np.abs(g - g64) <= 1e-4 * scale + 1e-6)
    # central difference in float64 (quadratic loss: no truncation term)
    v = synth.rng_for("fd-dir").standard_normal((h, w))
    eps = 1e-3

    def L(z):
        Fz = oracle.full(z)
        return float(np.sum(Wt.astype(np.float64) * Fz * Fz))
    fd = (L(x.astype(np.float64) + eps * v) - L(x.astype(np.float64) - eps * v)) / (2 * eps)
    assert abs(fd - float(np.sum(g * v))) <= 1e-4 * abs(fd) + 1e-3


def test_gradcheck_tiny():
    torch.manual_seed(0)
    x = torch.randn(6, 5, device="cuda", dtype=torch.float32, requires_grad=True)

    # float32 kernels: compare analytic vs numerical jacobian-vector products loosely
    def f(z):
        return fht.FHTFunction.apply(z)
    y = f(x)
    gy = torch.randn_like(y)
    (gx,) = torch.autograd.grad(y, x, gy)
    # <J^T gy, v> vs <gy, J v> with J v = F(v) (linear map)
    v = torch.randn_like(x).detach()
    lhs = float((gx.double() * v.double()).sum())
    with torch.no_grad():
        rhs = float((gy.double() * f(v).double()).sum())
    assert abs(lhs - rhs) <= 1e-4 * max(1.0, abs(lhs))


@pytest.mark.parametrize("h,w,shifted", [(300, 520, False), (1000, 70, False), (129, 257, True)])
def test_adjoint_ignores_cells_that_reach_no_pixel(h, w, shifted):
    # Cells whose pattern holds no image pixel (the forward of an all-ones
    # image is 0 there) cannot reach the image gradient.  The adjoint reads
    # the structurally zero part of them as zero; huge values there must not
    # change one bit of the float32 gradient.
    ones = oracle.full(np.ones((h, w)))
    if shifted:
        ones = oracle.fhtshift_full(ones, w, h)
    mask = ones == 0
    assert mask.any()
    rng = np.random.default_rng(5)
    g = rng.standard_normal(ones.shape).astype(np.float32)
    g2 = g.copy()
    g2[mask] = 3.0e38
    a = host(P.adjoint(dev(g), w, h, shifted=shifted))
    b = host(P.adjoint(dev(g2), w, h, shifted=shifted))
    assert np.array_equal(a, b)
    assert np.all(np.isfinite(b))
