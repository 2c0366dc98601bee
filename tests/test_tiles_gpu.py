"""Every forward parity case on both tile heights of the pass kernels.

Passes of at most 5 stages run on 32-row tiles (4 waves) or 64-row tiles
(8 waves); the default rule picks one per stage count.  This module reruns
the forward, max-transform, range and batch parity tests with every stage
count forced to each height in turn, so both kernels are checked against the
oracle whatever the default is (the 512-image batch against the single-image
path at the same height; its per-image oracle comparison runs once, at the
default rule, in test_batch_gpu).  Results must not depend on the height (the
same additions in the same order).
"""
import pytest

from test_batch_gpu import (batch512, test_batch512_matches_single_image_path,  # noqa: F401
                            test_batch_graph_replay, test_batch_quadrant_subsets,
                            test_batch_with_tiny_sides_matches_oracle, test_small_batch_matches_oracle)
from test_forward_gpu import *  # noqa: F401,F403
from test_max_gpu import *  # noqa: F401,F403
from test_range_gpu import test_range_any_pieces, test_range_scaled  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True, params=[32, 64], ids=["rows32", "rows64"])
def forced_tile_rows(request):
    from paper_1811_06378_amd import fht

    for k in range(3, 17):
        fht.set_tile_rows(k, request.param)
    yield request.param
    for k in range(3, 17):
        fht.set_tile_rows(k, None)
