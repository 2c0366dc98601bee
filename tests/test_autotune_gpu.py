"""Stage-fusion depth on the GPU: every split of the stages into passes gives
bit-identical results (the additions of a stage do not depend on how stages
are grouped), and the autotuner keeps a valid split whose results still
match the oracle.  The process-wide split is restored after each test."""
import numpy as np
import pytest
import torch

import oracle
import gpu_util as P
from gpu_util import assert_equal, dev, host
from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("side,k,splits", [(512, 9, [[4, 5], [6, 3], [3, 6]]), (1024, 10, [[6, 4], [4, 6]]),
                                           (2048, 11, [[5, 6]])])
def test_every_split_is_bit_identical(side, k, splits):
    img = synth.random_image(side, side, "f32", seed=k)
    x = dev(img)
    ref = P.forward(x).clone()
    try:
        for sp in splits:
            fht.set_pass_split(k, sp)
            assert torch.equal(P.forward(x), ref), sp
            G = P.adjoint(ref, side, side)
            fht.set_pass_split(k, None)
            assert torch.equal(G, P.adjoint(ref, side, side)), sp
    finally:
        fht.set_pass_split(k, None)


def test_autotune_keeps_parity():
    h, w = 300, 700          # k = 9 and 10
    try:
        sh, sw = fht.autotune(w, h, torch.uint8, reps=5)
        assert sum(sh) == 9 and sum(sw) == 10
        assert all(3 <= g <= 6 for g in sh + sw)
        img = synth.random_image(h, w, "u8", seed=5)
        assert_equal(host(P.forward(dev(img))).astype(np.float64), oracle.full(img), "after autotune")
    finally:
        fht.set_pass_split(9, None)
        fht.set_pass_split(10, None)
