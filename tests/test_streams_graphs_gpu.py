"""System behaviour on the GPU: calls on a non-default stream, capture of
the single-image forward and adjoint in a HIP graph (replayed several
times with eager work in between, every replay checked against the eager
result), batch workspace validation, and an int32 batch."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_equal, dev, host
from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu


def test_forward_on_a_side_stream():
    img = synth.random_image(300, 520, "f32", seed=1)
    x = dev(img)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        H = fht.forward(x)
        G = fht.adjoint(H, 520, 300)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    assert_equal(host(H).astype(np.float64), oracle.full(img.astype(np.float64), single=True), "side stream fwd")
    assert torch.equal(G, fht.adjoint(fht.forward(x), 520, 300))


@pytest.mark.parametrize("h,w", [(300, 520), (1024, 1024)])
def test_forward_adjoint_graph_replay(h, w):
    img = synth.random_image(h, w, "f32", seed=2)
    x = dev(img)
    rows, cols = fht.hough_shape(w, h)
    H = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
    G = torch.empty((h, w), dtype=torch.float32, device="cuda")
    ws = torch.empty(max(fht.workspace_size(w, h), 256), dtype=torch.uint8, device="cuda")
    wsa = torch.empty(max(fht.adjoint_workspace_size(w, h), 256), dtype=torch.uint8, device="cuda")

    def step():
        fht.forward(x, out=H, workspace=ws)
        fht.adjoint(H, w, h, out=G, workspace=wsa)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    H_ref, G_ref = H.clone(), G.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        H.fill_(-7.0)
        G.fill_(-7.0)
        _ = torch.randn(4096, device="cuda").cumsum(0)   # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(H, H_ref) and torch.equal(G, G_ref), rep


def test_batch_workspace_validation():
    plan = fht.BatchPlan([(40, 50), (70, 30)], in_dtype=torch.uint8)
    xs = [dev(synth.random_image(40, 50, "u8")), dev(synth.random_image(70, 30, "u8"))]
    table = plan.pointer_table(xs)
    packed = plan.output()
    L = fht.lib()
    # too small
    rc = L.fht_batch_forward(plan._plan, table.data_ptr(), packed.data_ptr(), plan.workspace.data_ptr(),
                             plan.workspace_bytes - 1, fht._stream())
    assert rc == fht.FHT_ERR_WORKSPACE
    # misaligned
    big = torch.empty(plan.workspace_bytes + 512, dtype=torch.uint8, device="cuda")
    rc = L.fht_batch_forward(plan._plan, table.data_ptr(), packed.data_ptr(), big.data_ptr() + 4,
                             plan.workspace_bytes, fht._stream())
    assert rc == fht.FHT_ERR_INVALID
    with pytest.raises(ValueError):
        plan.pointer_table([xs[1], xs[0]])


def test_batch_int32():
    sizes = [(13, 40), (64, 64), (100, 37), (129, 257)]
    imgs = [synth.random_image(h, w, "i32", seed=i) for i, (h, w) in enumerate(sizes)]
    plan = fht.BatchPlan(sizes, in_dtype=torch.int32)
    views = plan([dev(x) for x in imgs])
    torch.cuda.synchronize()
    for x, v in zip(imgs, views):
        assert_equal(host(v).astype(np.float64), oracle.full(x.astype(np.float64)), "batch i32 %s" % (x.shape,))
