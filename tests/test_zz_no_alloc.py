"""The allocation-free forward (fht_forward_noalloc) against fht_forward.

Both entry points run the same pass kernels; the allocation-free one keeps
its bands in the library's per-device scratch array.  Each case makes two
calls in a row, the second on a smaller image, so the second runs on scratch
that still holds the first call's bands; every output is poisoned before the
call and must equal fht_forward's result bit for bit (and the oracle's on
the small images).
"""
import numpy as np
import pytest
import torch

from gpu_util import assert_equal, dev, host, poisoned, poisoned_ws

pytestmark = pytest.mark.gpu


def _fht():
    from paper_1811_06378_amd import fht
    return fht


def _out_dtype(t):
    return torch.float32 if t == torch.float32 else torch.int32


def _both(x, quads="full", shifted=False, op="sum"):
    fht = _fht()
    h, w = x.shape
    shape = fht.hough_shape(w, h, quads)
    ref = fht.forward(x, quads, shifted, out=poisoned(shape, _out_dtype(x.dtype)),
                      workspace=poisoned_ws(fht.workspace_size(w, h, quads, x.dtype)), op=op)
    got = fht.forward_noalloc(x, poisoned(shape, _out_dtype(x.dtype)), quads, shifted, op=op)
    return host(got), host(ref)


def _image(h, w, kind, seed):
    from paper_1811_06378_amd import synth
    return synth.random_image(h, w, kind, seed=seed)


# (first call, second call): (h, w, kind, quads, shifted, op); the second image is smaller
CASES = [
    ((1024, 2048, "f32", "full", False, "sum"), (300, 517, "f32", "full", False, "sum")),
    ((1000, 1000, "u8", "full", True, "sum"), (129, 64, "u8", "full", True, "sum")),
    ((777, 1500, "i32", "full", False, "max"), (61, 90, "i32", "full", False, "max")),
    ((900, 640, "f32", (1, 3), False, "sum"), (5, 3, "f32", "full", False, "sum")),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_equals_forward_twice(first, second, oracle_mod):
    torch.cuda.set_device(0)
    for i, (h, w, kind, quads, shifted, op) in enumerate((first, second)):
        x = dev(_image(h, w, kind, seed=10 + i))
        got, ref = _both(x, quads, shifted, op)
        assert_equal(got, ref, "noalloc vs fht_forward, call %d (%dx%d %s)" % (i + 1, h, w, kind))
        if i == 1:
            img = _image(h, w, kind, seed=10 + i)
            if quads == "full" and op == "sum":
                want = oracle_mod.full(img, single=(kind == "f32"))
                if shifted:
                    want = oracle_mod.fhtshift_full(want, w, h)
                assert_equal(got.astype(np.float64), want, "noalloc vs oracle")


def test_noalloc_rejects_transforms_beyond_its_scratch():
    fht = _fht()
    torch.cuda.set_device(0)
    x = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda")
    assert fht.workspace_size(2048, 2048, "full", torch.float32) > fht.NOALLOC_SCRATCH_BYTES
    out = poisoned(fht.hough_shape(2048, 2048), torch.float32)
    with pytest.raises(ValueError, match="allocation-free"):
        fht.forward_noalloc(x, out)
    # nothing was launched: the output still holds the poison
    assert torch.isnan(out).all().item()
    # the next call that fits still works
    y = dev(_image(64, 48, "f32", seed=3))
    got, ref = _both(y)
    assert_equal(got, ref, "noalloc after a rejected call")
