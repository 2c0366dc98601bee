"""Stacks of same-size images: batch_forward (one batch plan for the whole
stack) and batch_adjoint (images spread over side streams), and the autograd
wrapper that uses them.  Every result must equal the single-image path bit for
bit (the same kernels and add order), and the single-image path is pinned to
the oracle elsewhere; one image per case is also checked against the oracle
here."""
import numpy as np
import pytest
import torch

import oracle
import gpu_util as P
from gpu_util import dev, host
from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu


def _stack(n, h, w, kind, seed=0):
    return np.stack([synth.random_image(h, w, kind, seed=seed + i) for i in range(n)])


@pytest.mark.parametrize("n,h,w,kind", [(5, 100, 130, "f32"), (3, 64, 64, "u8"), (4, 37, 300, "i32"),
                                        (2, 4, 9, "f32"), (1, 50, 60, "f32")])
def test_batch_forward_equals_single(n, h, w, kind):
    imgs = _stack(n, h, w, kind, seed=3)
    x = dev(imgs)
    got = fht.batch_forward(x)
    for i in range(n):
        assert torch.equal(got[i], P.forward(x[i]))
    np.testing.assert_array_equal(host(got[0]).astype(np.float64),
                                  oracle.full(imgs[0].astype(np.float64), single=(kind == "f32")))


def test_batch_forward_shifted_and_quadrants():
    imgs = _stack(3, 90, 70, "f32", seed=5)
    x = dev(imgs)
    got = fht.batch_forward(x, shifted=True)
    for i in range(3):
        assert torch.equal(got[i], P.forward(x[i], shifted=True))
    got_q = fht.batch_forward(x, quads=[2, 3])
    for i in range(3):
        assert torch.equal(got_q[i], P.forward(x[i], quads=[2, 3]))


def test_batch_forward_reuses_plan_with_new_data():
    a = dev(_stack(4, 80, 96, "f32", seed=1))
    b = dev(_stack(4, 80, 96, "f32", seed=9))
    ra = fht.batch_forward(a)
    rb = fht.batch_forward(b)
    for i in range(4):
        assert torch.equal(ra[i], P.forward(a[i]))
        assert torch.equal(rb[i], P.forward(b[i]))


@pytest.mark.parametrize("streams", [1, 2, 3])
@pytest.mark.parametrize("n", [1, 3, 4, 5, 9])
def test_batch_adjoint_equals_single(n, streams):
    # one launch per pass kind over the stack; with streams > 1 the stack is
    # split over side streams once it has 2 images per stream
    h, w = 120, 75
    rows, cols = fht.hough_shape(w, h)
    rng = np.random.default_rng(n * 10 + streams)
    g = dev(rng.standard_normal((n, rows, cols)).astype(np.float32))
    got = P.batch_adjoint(g, w, h, streams=streams)
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(got[i], P.adjoint(g[i], w, h))
    np.testing.assert_allclose(host(got[0]).astype(np.float64),
                               oracle.adjoint_full(host(g[0]).astype(np.float64), w, h), rtol=1e-4, atol=1e-3)


def test_batch_adjoint_groups_of_large_images():
    """4096^2 gradients: a group holds as many images as keep their bands
    within 2 GiB (7), so 9 images run as groups of 7 and 2 reusing one
    workspace; every image equals the single-image adjoint bit for bit."""
    h = w = 4096
    rows, cols = fht.hough_shape(w, h)
    n = 9
    one = (fht.adjoint_workspace_size(w, h) + 255) // 256 * 256
    assert fht.adjoint_stack_workspace_size(w, h, n) == ((2 << 30) // one) * one < n * one
    g = torch.empty((n, rows, cols), device="cuda").normal_(generator=torch.Generator(device="cuda").manual_seed(9))
    got = P.batch_adjoint(g, w, h)
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(got[i], P.adjoint(g[i], w, h)), "image %d" % i
    del g, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("quads,shifted", [([2, 3], False), ([1], False), ("full", True)])
def test_batch_adjoint_subsets_shifted_and_strides(quads, shifted):
    h, w = 70, 140
    rows, cols = fht.hough_shape(w, h, quads)
    rng = np.random.default_rng(8)
    big = dev(rng.standard_normal((10, rows, cols + 3)).astype(np.float32))
    g = big[::2, :, :cols]  # image stride 2 * rows * (cols + 3), row pitch cols + 3
    out_big = torch.full((5, h + 2, w + 5), -1.0, device="cuda")
    out = out_big[:, :h, :w]
    fht.batch_adjoint(g, w, h, quads=quads, shifted=shifted, out=out)
    for i in range(5):
        assert torch.equal(out[i], P.adjoint(g[i].contiguous(), w, h, quads=quads, shifted=shifted))
    assert bool(torch.all(out_big[:, h:, :] == -1.0)) and bool(torch.all(out_big[:, :, w:] == -1.0))


@pytest.mark.parametrize("h,w", [(3, 6), (1, 1), (2, 9), (4, 4), (1, 40), (40, 2)])
def test_batch_adjoint_tiny_quadrants(h, w):
    # sides up to 4: direct kernels inside the stack (the image index on the grid)
    rows, cols = fht.hough_shape(w, h)
    g = dev(np.random.default_rng(3 + h * w).standard_normal((5, rows, cols)).astype(np.float32))
    got = P.batch_adjoint(g, w, h)
    for i in range(5):
        assert torch.equal(got[i], P.adjoint(g[i], w, h))


def test_batch_adjoint_int32_exact():
    h, w = 66, 130
    rows, cols = fht.hough_shape(w, h)
    rng = np.random.default_rng(2)
    g = rng.integers(-1000, 1000, (3, rows, cols)).astype(np.int32)
    got = host(P.batch_adjoint(dev(g), w, h))
    for i in range(3):
        np.testing.assert_array_equal(got[i].astype(np.float64), oracle.adjoint_full(g[i].astype(np.float64), w, h))


@pytest.mark.parametrize("n", [3, 6])
def test_autograd_on_a_stack(n):
    h, w = 64, 80
    imgs = _stack(n, h, w, "f32", seed=21)
    x = dev(imgs).requires_grad_()
    rows, cols = fht.hough_shape(w, h)
    wt = dev(np.random.default_rng(4).random((n, rows, cols)).astype(np.float32))
    H = fht.fht(x)
    loss = (wt * H * H).sum()
    loss.backward()
    gH = (2 * wt * H).detach()
    for i in range(n):
        assert torch.equal(H[i].detach(), P.forward(x[i].detach()))
        assert torch.equal(x.grad[i], P.adjoint(gH[i].contiguous(), w, h))
