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


# ------------------------------------------------------------ poisoned outputs
#
# Every parity call writes into buffers pre-filled with a sentinel that no
# correct result holds (NaN in float32, 0x7FFFFFFF in int32), and its
# workspace is filled with 0xFF bytes (NaN / -1 in every band cell), so a
# cell the kernels never write, or a band cell they read without writing it
# first, cannot pass by holding an earlier result.
SENTINEL_I32 = 0x7FFFFFFF


def poisoned(shape, dtype) -> torch.Tensor:
    t = torch.empty(shape, dtype=dtype, device="cuda")
    if dtype == torch.float32:
        t.fill_(float("nan"))
    elif dtype == torch.int32:
        t.fill_(SENTINEL_I32)
    else:
        t.fill_(0xFF)
    return t


def poisoned_ws(nbytes: int) -> torch.Tensor:
    return torch.full((max(int(nbytes), 256),), 0xFF, dtype=torch.uint8, device="cuda")


def _out_dtype(t):
    return torch.float32 if t == torch.float32 else torch.int32


def _fht():
    from paper_1811_06378_amd import fht
    return fht


def forward(x, quads="full", shifted=False, op="sum"):
    fht = _fht()
    h, w = x.shape
    out = poisoned(fht.hough_shape(w, h, quads), _out_dtype(x.dtype))
    ws = poisoned_ws(fht.workspace_size(w, h, quads, x.dtype))
    return fht.forward(x, quads, shifted, out=out, workspace=ws, op=op)


def adjoint(g, w, h, quads="full", shifted=False):
    fht = _fht()
    out = poisoned((h, w), g.dtype)
    ws = poisoned_ws(fht.adjoint_workspace_size(w, h, quads, g.dtype))
    return fht.adjoint(g, w, h, quads, shifted, out=out, workspace=ws)


def range_transform(x, S1, S, transposed=False):
    fht = _fht()
    h, w = x.shape
    out = poisoned(fht.range_shape(w, h, S1, S, transposed), _out_dtype(x.dtype))
    ws = poisoned_ws(fht.range_workspace_size(w, h, S1, S, transposed, x.dtype))
    return fht.range_transform(x, S1, S, transposed, out=out, workspace=ws)


def range_scaled(x, num, den, S1, S, transposed=False):
    fht = _fht()
    h, w = x.shape
    out = poisoned(fht.range_scaled_shape(w, h, num, den, S1, S, transposed), _out_dtype(x.dtype))
    ws = poisoned_ws(fht.range_scaled_workspace_size(w, h, num, den, S1, S, transposed, x.dtype))
    return fht.range_scaled(x, num, den, S1, S, transposed, out=out, workspace=ws)


def range_adjoint(g, w, h, S1, S, transposed=False):
    fht = _fht()
    out = poisoned((h, w), g.dtype)
    ws = poisoned_ws(fht.range_adjoint_workspace_size(w, h, S1, S, transposed, g.dtype))
    return fht.range_adjoint(g, w, h, S1, S, transposed, out=out, workspace=ws)


def shift(H, w, h, inverse=False):
    fht = _fht()
    return fht.shift(H, w, h, inverse, out=poisoned(tuple(H.shape), H.dtype))


def batch_adjoint(g, w, h, quads="full", shifted=False, streams=1):
    fht = _fht()
    out = poisoned((g.shape[0], h, w), g.dtype)
    return fht.batch_adjoint(g, w, h, quads, shifted, out=out, streams=streams)


def batch_run(plan, imgs):
    """One batched forward into a poisoned packed buffer with a poisoned
    workspace; returns the per-image views."""
    packed = poisoned((plan.out_elems,), plan.out_dtype)
    plan.run(plan.pointer_table(imgs), packed, workspace=poisoned_ws(plan.workspace_bytes))
    return plan.views(packed)
