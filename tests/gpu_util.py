"""Helpers for the GPU parity tests: device transfer and the tolerance rule."""
from __future__ import annotations

import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


# Float tolerance.  The FP32 kernels add binary32 values in the stage order of
# the recurrence; each output is a sum of n terms formed by log2(n) rounded
# additions, so |H32 - H64| <= log2(n) * 2^-24 * FHT(|I|) (about 7e-7 relative
# at n = 4096).  The bar is 1e-5 relative to the sum of magnitudes, so that
# cancellation in signed data does not inflate a relative error.
REL_TOL = 1e-5


def assert_close_fp(got: np.ndarray, ref64: np.ndarray, absref64: np.ndarray, what: str = ""):
    err = np.abs(got.astype(np.float64) - ref64)
    bound = REL_TOL * absref64 + 1e-30
    bad = err > bound
    if np.any(bad):
        i = np.argwhere(bad)[0]
        raise AssertionError("%s: %d cells exceed 1e-5*FHT(|I|); first %s got %r want %r (bound %r)"
                             % (what, int(bad.sum()), tuple(i), got[tuple(i)], ref64[tuple(i)], bound[tuple(i)]))


def assert_equal(got: np.ndarray, want: np.ndarray, what: str = ""):
    if got.shape != want.shape:
        raise AssertionError("%s: shape %s != %s" % (what, got.shape, want.shape))
    neq = got != want
    if np.any(neq):
        i = np.argwhere(neq)[0]
        raise AssertionError("%s: %d of %d cells differ; first %s got %r want %r"
                             % (what, int(neq.sum()), neq.size, tuple(i), got[tuple(i)], want[tuple(i)]))
