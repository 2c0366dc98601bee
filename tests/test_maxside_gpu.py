"""The largest side the library accepts (65536), on a thin image so the full
Hough image (131085 x 65544 int32, 34 GB) still fits: sampled cells against
the oracle's direct pattern sums, every row summing to the image total, and
the standalone fhtshift (more rows than one grid dimension holds) against
the oracle's rolls on sampled rows."""
import numpy as np
import pytest
import torch

import oracle
import gpu_util as P
from gpu_util import dev
from paper_1811_06378_amd import fht, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("h,w", [(5, 65536), (65536, 5)])
def test_max_side_forward_and_shift(h, w):
    img = synth.random_image(h, w, "u8", seed=65)
    x = dev(img)
    H = P.forward(x)
    rows, cols = H.shape
    assert (rows, cols) == fht.hough_shape(w, h) == (131085, 65544)
    rng = np.random.default_rng(1)
    rr = rng.integers(0, rows, 1500)
    cc = rng.integers(0, cols, 1500)
    got = H[torch.from_numpy(rr).cuda(), torch.from_numpy(cc).cuda()].cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(got, oracle.full_cells(img, rr, cc))
    total = int(img.astype(np.int64).sum())
    rs = H.sum(dim=1, dtype=torch.int64)
    assert bool(torch.all(rs == total))
    S = fht.shift(H, w, h)
    hp, wp = 1 << (h - 1).bit_length(), 1 << (w - 1).bit_length()
    for r in list(rng.integers(0, rows, 12)) + [0, rows - 1, 65535, 65536]:
        q, s = oracle.row_quadrant(w, h, int(r))
        roll = oracle.fhtshift_roll(q, hp, wp, s)
        np.testing.assert_array_equal(S[int(r)].cpu().numpy(), np.roll(H[int(r)].cpu().numpy(), roll))
    del H, S
    torch.cuda.empty_cache()
