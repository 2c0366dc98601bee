"""Batched forward on the GPU: many images of different sizes in one plan,
per image bit-exact against the oracle (all 512 images of the 512-image
workload) and identical to the single-image path; outputs and workspaces
are poisoned before every call; the batched call replays correctly from a
captured HIP graph."""
import numpy as np
import pytest
import torch

import oracle
import gpu_util as P
from gpu_util import assert_equal, dev, host
from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu

SMALL = [(5, 5), (8, 8), (13, 40), (64, 64), (100, 37), (129, 257), (300, 520), (520, 300), (7, 1000), (1000, 9),
         (256, 256), (65, 65)]


def _run(plan, imgs):
    xs = [dev(x) for x in imgs]
    views = P.batch_run(plan, xs)
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


TINY = [(1, 1), (1, 7), (7, 1), (2, 3), (3, 2), (4, 4), (2, 100), (100, 3), (4, 37), (5, 5), (64, 64), (1, 300)]


@pytest.mark.parametrize("kind", ["u8", "i32", "f32"])
def test_batch_with_tiny_sides_matches_oracle(kind):
    """Sides 1..4 (quadrants of at most 4 rows run as direct cells inside the
    plan) mixed with ordinary images: every image bit-exact."""
    imgs = [synth.random_image(h, w, kind, seed=30 + i) for i, (h, w) in enumerate(TINY)]
    dt = {"u8": torch.uint8, "i32": torch.int32, "f32": torch.float32}[kind]
    plan = fht.BatchPlan(TINY, in_dtype=dt)
    for (h, w), x, got in zip(TINY, imgs, _run(plan, imgs)):
        want = oracle.full(x.astype(np.float64), single=(kind == "f32"))
        assert_equal(got.astype(np.float64), want, "tiny batch %s %dx%d" % (kind, h, w))
    plan_q = fht.BatchPlan(TINY, quads=[2, 4], in_dtype=dt)
    for x, got in zip(imgs, _run(plan_q, imgs)):
        assert_equal(got.astype(np.float64), oracle.stacked_quadrants(x.astype(np.float64), [2, 4],
                                                                       single=(kind == "f32")), "tiny batch q2,q4")


@pytest.mark.parametrize("quads", [[1], [2, 3], [4]])
def test_batch_quadrant_subsets(quads):
    sizes = SMALL[:8]
    imgs = [synth.random_image(h, w, "u8", seed=i) for i, (h, w) in enumerate(sizes)]
    plan = fht.BatchPlan(sizes, quads=quads, in_dtype=torch.uint8)
    for x, got in zip(imgs, _run(plan, imgs)):
        assert_equal(got.astype(np.float64), oracle.stacked_quadrants(x, quads), "batch quads %s" % quads)


@pytest.fixture(scope="module")
def batch512():
    """The 512-image workload (sides uniform in 64..2048, uint8, about 38 GB
    of int32 Hough images) through one plan, into a poisoned packed buffer
    with a poisoned workspace."""
    sizes = synth.batch_sizes(0)
    plan = fht.BatchPlan(sizes, in_dtype=torch.uint8)
    imgs = synth.batch512(0)
    xs = [dev(x) for x in imgs]
    views = P.batch_run(plan, xs)
    torch.cuda.synchronize()
    yield imgs, xs, views
    del views, xs, plan
    torch.cuda.empty_cache()


BATCH_CHUNKS = 8


@pytest.mark.slow
@pytest.mark.parametrize("chunk", range(BATCH_CHUNKS))
def test_batch512_every_image_matches_oracle(batch512, chunk):
    """Every one of the 512 batched Hough images equals the oracle bit for
    bit (streamed one image at a time; eight chunks of 64 images)."""
    imgs, _, views = batch512
    per = len(imgs) // BATCH_CHUNKS
    for i in range(chunk * per, (chunk + 1) * per):
        assert_equal(host(views[i]).astype(np.float64), oracle.full(imgs[i]),
                     "batch512 image %d %s" % (i, imgs[i].shape))


def test_batch512_matches_single_image_path(batch512):
    """Every batched Hough image also equals the single-image forward."""
    _, xs, views = batch512
    for i, (x, v) in enumerate(zip(xs, views)):
        assert torch.equal(v, P.forward(x)), "image %d (%s) differs from the single-image path" % (i, tuple(x.shape))


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


@pytest.mark.parametrize("kind,n,h,w", [("u8", 5, 100, 37), ("f32", 3, 129, 64), ("i32", 4, 3, 70), ("f32", 1, 1, 1)])
def test_stack_entry_matches_oracle_and_pointer_table(kind, n, h, w):
    """fht_batch_forward_stack (image i at base + i * stride, resolved on the
    device): every image bit-exact against the oracle and identical to the
    pointer-table call, into poisoned outputs and workspaces; a stride larger
    than one image (a sliced stack) works the same."""
    dt = {"u8": torch.uint8, "i32": torch.int32, "f32": torch.float32}[kind]
    imgs = [synth.random_image(h, w, kind, seed=70 + i) for i in range(n)]
    plan = fht.BatchPlan([(h, w)] * n, in_dtype=dt)
    x = torch.stack([dev(a) for a in imgs])
    packed = P.poisoned((plan.out_elems,), plan.out_dtype)
    plan.run_stack(x, packed, workspace=P.poisoned_ws(plan.workspace_bytes))
    ref = P.batch_run(plan, [x[i] for i in range(n)])
    for i, (a, v) in enumerate(zip(imgs, plan.views(packed))):
        assert torch.equal(v, ref[i]), "stack image %d differs from the pointer-table call" % i
        want = oracle.full(a.astype(np.float64), single=(kind == "f32"))
        assert_equal(host(v).astype(np.float64), want, "stack %s image %d" % (kind, i))
    # every other image of a 2n stack: stride of two images
    big = torch.stack([x[i // 2] for i in range(2 * n)])[::2]
    assert big.stride(0) == 2 * h * w
    packed2 = P.poisoned((plan.out_elems,), plan.out_dtype)
    rc = fht.lib().fht_batch_forward_stack(plan._plan, big.data_ptr(), big.stride(0) * big.element_size(),
                                           packed2.data_ptr(), plan.workspace.data_ptr(), plan.workspace.numel(),
                                           fht._stream())
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(packed2, packed)


def test_stack_entry_graph_replay_and_rejections():
    n, h, w = 6, 300, 200
    x = torch.stack([dev(synth.random_image(h, w, "f32", seed=80 + i)) for i in range(n)])
    plan = fht.BatchPlan([(h, w)] * n, in_dtype=torch.float32)
    eager = plan.output()
    plan.run_stack(x, eager)
    torch.cuda.synchronize()
    packed = plan.output()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run_stack(x, packed)
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(g):
        plan.run_stack(x, packed)
    for rep in range(3):
        packed.fill_(-1.0)
        _ = torch.randn(1000, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(packed, eager), "replay %d differs" % rep
    del g
    L = fht.lib()
    ws = plan.workspace
    # a stride shorter than one image, and a plan of unequal sizes, are rejected before any launch
    assert L.fht_batch_forward_stack(plan._plan, x.data_ptr(), h * w * 4 - 4, packed.data_ptr(), ws.data_ptr(),
                                     ws.numel(), fht._stream()) == fht.FHT_ERR_INVALID
    mixed = fht.BatchPlan([(h, w), (h, w + 1)], in_dtype=torch.float32)
    out = mixed.output()
    assert L.fht_batch_forward_stack(mixed._plan, x.data_ptr(), h * w * 4, out.data_ptr(), mixed.workspace.data_ptr(),
                                     mixed.workspace.numel(), fht._stream()) == fht.FHT_ERR_INVALID
    with pytest.raises(ValueError):
        mixed.run_stack(x[:2], out)
