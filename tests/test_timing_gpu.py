"""Launch timing (fht_timing_enable / fht_timing_report): the per-kernel HIP
events that the benchmark's roofline figure is computed from."""
import numpy as np
import pytest
import torch

from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu


def _forward(img, reps):
    out = None
    for _ in range(reps):
        out = fht.forward(img)
    torch.cuda.synchronize()
    return out


def test_forward_launches_are_counted_per_kernel():
    img = torch.from_numpy(synth.random_image(1024, 1024, "f32", seed=1)).cuda()
    _forward(img, 1)
    fht.timing_enable(True)
    try:
        _forward(img, 3)
    finally:
        fht.timing_enable(False)
    rep = fht.timing_report()
    # 1024: two passes (GB = stages - 3), the first from the image, the last to
    # the Hough image; 6-stage passes run 8 waves, shorter ones tile_rows / 8
    g1, g2 = fht.pass_split(1024)

    def waves(g):
        return 8 if g == 6 else fht.tile_rows(1024) // 8

    first = "fht::fht_pass_kernel<float, float, %d, true, false, 0, %d, 0>" % (g1 - 3, waves(g1))
    last = "fht::fht_pass_kernel<float, float, %d, false, true, 0, %d, 0>" % (g2 - 3, waves(g2))
    assert set(rep) == {first, last}, rep
    for name in (first, last):
        launches, total_ms = rep[name]
        assert launches == 3
        assert 0.0 < total_ms / launches < 50.0


def test_enable_clears_and_disable_stops_recording():
    img = torch.from_numpy(synth.random_image(300, 200, "u8", seed=2)).cuda()
    fht.timing_enable(True)
    _forward(img, 2)
    fht.timing_enable(True)  # starts over
    _forward(img, 1)
    fht.timing_enable(False)
    _forward(img, 4)  # not recorded
    rep = fht.timing_report()
    assert rep and all(n == 1 for n, _ in rep.values()), rep


def test_timing_does_not_change_results():
    img = torch.from_numpy(synth.random_image(517, 389, "f32", seed=3)).cuda()
    ref = _forward(img, 1).cpu()
    fht.timing_enable(True)
    try:
        got = _forward(img, 1).cpu()
    finally:
        fht.timing_enable(False)
    assert torch.equal(ref, got)


def test_nothing_recorded_under_graph_capture():
    sizes = [(100, 90), (64, 200)]
    imgs = [torch.from_numpy(synth.random_image(h, w, "u8", seed=i)).cuda() for i, (h, w) in enumerate(sizes)]
    plan = fht.BatchPlan(sizes, in_dtype=torch.uint8)
    table = plan.pointer_table(imgs)
    packed = plan.output()
    plan.run(table, packed)
    torch.cuda.synchronize()
    want = packed.clone()
    fht.timing_enable(True)
    try:
        g = plan.capture(table, packed)  # one eager warm-up run, then the capture
        torch.cuda.synchronize()
        eager = sum(n for n, _ in fht.timing_report().values())
        packed.zero_()
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(packed, want)
    finally:
        fht.timing_enable(False)
    rep = fht.timing_report()
    # only the eager warm-up launches were recorded; replays add none
    assert sum(n for n, _ in rep.values()) == eager > 0
    del g
    np.testing.assert_array_equal(packed.cpu().numpy(), want.cpu().numpy())


def test_filter_records_only_matching_kernels():
    img = torch.from_numpy(synth.random_image(1024, 1024, "f32", seed=4)).cuda()
    g2 = fht.pass_split(1024)[-1]
    last = "fht::fht_pass_kernel<float, float, %d, false, true, 0, %d, 0>" % (
        g2 - 3, 8 if g2 == 6 else fht.tile_rows(1024) // 8)
    fht.timing_filter("%d, false, true, 0, " % (g2 - 3))
    fht.timing_enable(True)
    try:
        _forward(img, 2)
    finally:
        fht.timing_enable(False)
        fht.timing_filter(None)
    rep = fht.timing_report()
    assert list(rep) == [last] and rep[last][0] == 2, rep
    # the filter is cleared: both passes again
    fht.timing_enable(True)
    _forward(img, 1)
    fht.timing_enable(False)
    assert len(fht.timing_report()) == 2
