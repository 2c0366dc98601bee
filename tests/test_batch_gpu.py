"""Batched forward on the GPU: many images of different sizes in one plan,
per image bit-exact against the oracle and identical to the single-image
path; the batched call replays correctly from a captured HIP graph."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_equal, dev, host
from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu

SMALL = [(5, 5), (8, 8), (13, 40), (64, 64), (100, 37), (129, 257), (300, 520), (520, 300), (7, 1000), (1000, 9),
         (256, 256), (65, 65)]


def _run(plan, imgs):
    xs = [dev(x) for x in imgs]
    views = plan(xs)
    torch.cuda.synchronize()
    return [host(v) for v in views]


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_small_batch_matches_oracle(kind):
    imgs = [synth.random_image(h, w, kind, seed=i) for i, (h, w) in enumerate(SMALL)]
    dt = torch.uint8 if kind == "u8" else torch.float32
    plan = fht.BatchPlan(SMALL, in_dtype=dt)
    outs = _run(plan, imgs)
    for (h, w), x, got in zip(SMALL, imgs, outs):
        want = oracle.full(x.astype(np.float64), single=(kind == "f32"))
        assert_equal(got.astype(np.float64), want, "batch %s %dx%d" % (kind, h, w))


@pytest.mark.parametrize("quads", [[1], [2, 3], [4]])
def test_batch_quadrant_subsets(quads):
    sizes = SMALL[:8]
    imgs = [synth.random_image(h, w, "u8", seed=i) for i, (h, w) in enumerate(sizes)]
    plan = fht.BatchPlan(sizes, quads=quads, in_dtype=torch.uint8)
    for x, got in zip(imgs, _run(plan, imgs)):
        assert_equal(got.astype(np.float64), oracle.stacked_quadrants(x, quads), "batch quads %s" % quads)


def test_batch512_matches_single_image_path():
    """The 512-image workload (sides uniform in 64..2048): every batched Hough
    image equals the single-image forward bit for bit; six images are also
    checked against the oracle."""
    sizes = synth.batch_sizes(0)
    plan = fht.BatchPlan(sizes, in_dtype=torch.uint8)
    imgs = synth.batch512(0)
    xs = [dev(x) for x in imgs]
    packed = plan.output()
    plan.run(plan.pointer_table(xs), packed)
    views = plan.views(packed)
    for i, (x, v) in enumerate(zip(xs, views)):
        ref = fht.forward(x)
        assert torch.equal(v, ref), "image %d (%s) differs from the single-image path" % (i, tuple(x.shape))
    for i in (0, 1, 100, 255, 400, 511):
        assert_equal(host(views[i]).astype(np.float64), oracle.full(imgs[i]), "batch512 image %d" % i)


def test_batch_graph_replay():
    """Capture the batched call once; every replay (with eager work between
    replays) reproduces the eager result."""
    sizes = SMALL
    imgs = [synth.random_image(h, w, "f32", seed=10 + i) for i, (h, w) in enumerate(sizes)]
    plan = fht.BatchPlan(sizes, in_dtype=torch.float32)
    xs = [dev(x) for x in imgs]
    table = plan.pointer_table(xs)
    eager = plan.output()
    plan.run(table, eager)
    torch.cuda.synchronize()
    packed = plan.output()
    g = plan.capture(table, packed)
    for rep in range(3):
        packed.fill_(-1.0)
        _ = torch.randn(1000, device="cuda").sum()   # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(packed, eager), "replay %d differs" % rep
