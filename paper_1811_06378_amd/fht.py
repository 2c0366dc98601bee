"""Python binding of libfht.so (ctypes).  Argument marshalling only.

Every transform runs in the library's HIP kernels; torch supplies device
memory (tensors) and the current HIP stream.  If the library is missing the
calls raise instead of falling back to anything else.

Names follow the C ABI in include/fht.h:
  forward(img, quads='full', shifted=False, op='sum')
                                              sections 3.1, 3.3 (and 5; op='max': section 1)
  range_transform(img, S1, S, transposed)     section 4
  range_pieces / range_any(img, deg_lo, deg_hi) any inclination range, split into calls
  range_scaled(img, num, den, S1, S)          section 4 scale along the sheared axis
  shift(hough, w, h, inverse)                 section 5 (fhtshift)
  adjoint(grad, w, h, quads, shifted)         transpose of forward
  range_adjoint(grad, w, h, S1, S, transposed) transpose of range_transform; RangeFunction
  FHTFunction                                 autograd wrapper
  BatchPlan                                   batched forward (graph-capturable)
  cell_segment / peaks / detect_lines          Hough cell -> image segment (sections 3.2, 3.3)
  set_pass_split / autotune                   stage-fusion depth per pass (tuned on the device)
  timing_enable / timing_report               per-kernel launch times (HIP events)
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfht.so")

FHT_OK, FHT_ERR_INVALID, FHT_ERR_UNSUPPORTED, FHT_ERR_WORKSPACE, FHT_ERR_HIP, FHT_ERR_TIMEOUT = 0, -1, -2, -3, -4, -5
FHT_U8, FHT_I32, FHT_F32 = 0, 1, 2
FHT_Q1, FHT_Q2, FHT_Q3, FHT_Q4, FHT_FULL = 1, 2, 4, 8, 15
FHT_FLAG_SHIFTED, FHT_FLAG_MAX = 1, 2

_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_U = ctypes.c_uint
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PSZ = ctypes.POINTER(ctypes.c_size_t)
_PI32 = ctypes.POINTER(ctypes.c_int32)

# symbol -> (restype, argtypes); the full ABI of include/fht.h
SIGNATURES = {
    "fht_version": (_I, []),
    "fht_status_string": (ctypes.c_char_p, [_I]),
    "fht_last_error": (ctypes.c_char_p, []),
    "fht_hough_shape": (_I, [_I, _I, _U, _PI64, _PI64]),
    "fht_range_shape": (_I, [_I, _I, _I, _I, _I, _PI64, _PI64]),
    "fht_workspace_size": (_I, [_I, _I, _U, _I, _I, _PSZ]),
    "fht_range_workspace_size": (_I, [_I, _I, _I, _I, _I, _I, _I, _PSZ]),
    "fht_adjoint_workspace_size": (_I, [_I, _I, _U, _I, _PSZ]),
    "fht_forward": (_I, [_P, _I, _I, _I, _I64, _P, _I, _I64, _U, _U, _P, _SZ, _P]),
    "fht_forward_noalloc": (_I, [_P, _I, _I, _I, _I64, _P, _I, _I64, _U, _U, _P]),
    "fht_forward_stack_workspace_size": (_I, [_I, _I, _U, _I, _I, _I, _PSZ]),
    "fht_forward_stack": (_I, [_P, _I, _I, _I, _I64, _I64, _I, _P, _I, _I64, _I64, _U, _U, _P, _SZ, _P]),
    "fht_range": (_I, [_P, _I, _I, _I, _I64, _I, _I, _I, _P, _I, _I64, _P, _SZ, _P]),
    "fht_shift": (_I, [_P, _I64, _P, _I64, _I, _I, _I, _I, _P]),
    "fht_adjoint": (_I, [_P, _I, _I64, _P, _I64, _I, _I, _U, _U, _P, _SZ, _P]),
    "fht_adjoint_stack_workspace_size": (_I, [_I, _I, _U, _I, _I, _PSZ]),
    "fht_adjoint_stack": (_I, [_P, _I, _I64, _I64, _P, _I64, _I64, _I, _I, _I, _U, _U, _P, _SZ, _P]),
    "fht_batch_plan_create": (_I, [_PI32, _PI32, _I, _U, _I, _I, ctypes.POINTER(_P), _PSZ, _PI64, _PI64]),
    "fht_batch_forward": (_I, [_P, _P, _P, _P, _SZ, _P]),
    "fht_batch_forward_stack": (_I, [_P, _P, ctypes.c_int64, _P, _P, _SZ, _P]),
    "fht_batch_plan_destroy": (_I, [_P]),
    "fht_pass_split": (_I, [_I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "fht_range_scaled_shape": (_I, [_I, _I, _I, _I, _I, _I, _I, _PI64, _PI64]),
    "fht_range_scaled_workspace_size": (_I, [_I, _I, _I, _I, _I, _I, _I, _I, _I, _PSZ]),
    "fht_range_scaled": (_I, [_P, _I, _I, _I, _I64, _I, _I, _I, _I, _I, _P, _I, _I64, _P, _SZ, _P]),
    "fht_range_adjoint_workspace_size": (_I, [_I, _I, _I, _I, _I, _I, _PSZ]),
    "fht_range_adjoint": (_I, [_P, _I, _I64, _I, _I, _I, _P, _I64, _I, _I, _P, _SZ, _P]),
    "fht_cell_segment": (_I, [_I, _I, _U, _I64, _I64, _I, _PI32]),
    "fht_peaks": (_I, [_P, _I, _I64, _I64, _I64, _I, ctypes.c_double, _P, _I, _P, _P]),
    "fht_engine_status": (_I, [_P, _P]),
    "fht_set_tile_rows": (_I, [_I, _I]),
    "fht_tile_rows": (_I, [_I, ctypes.POINTER(_I)]),
    "fht_set_pass_split": (_I, [_I, _I, ctypes.POINTER(_I)]),
    "fht_autotune": (_I, [_I, _I, _I, _I, _I, _P]),
    "fht_timing_enable": (_I, [_I]),
    "fht_timing_filter": (_I, [ctypes.c_char_p]),
    "fht_timing_report": (_I, [_I, ctypes.c_char_p, _I, _PI64, ctypes.POINTER(ctypes.c_double)]),
}


class FHTError(RuntimeError):
    pass


def lib():
    """The loaded libfht.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise FHTError("libfht.so is not built (run python paper_1811_06378_amd/build.py); "
                               "there is no fallback path")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc == FHT_OK:
        return
    L = lib()
    msg = "%s: %s (%s)" % (what, L.fht_status_string(rc).decode(), L.fht_last_error().decode())
    if rc in (FHT_ERR_INVALID, FHT_ERR_UNSUPPORTED, FHT_ERR_WORKSPACE):
        raise ValueError(msg)
    raise FHTError(msg)


_QUADS = {"full": FHT_FULL, "q1": FHT_Q1, "q2": FHT_Q2, "q3": FHT_Q3, "q4": FHT_Q4}


def _quads(q) -> int:
    if isinstance(q, int):
        return q
    if isinstance(q, str):
        return _QUADS[q]
    m = 0
    for x in q:
        m |= 1 << (int(x) - 1)
    return m


def _dtypes(t: torch.dtype):
    if t == torch.uint8:
        return FHT_U8, FHT_I32, torch.int32
    if t == torch.int32:
        return FHT_I32, FHT_I32, torch.int32
    if t == torch.float32:
        return FHT_F32, FHT_F32, torch.float32
    raise ValueError("unsupported image dtype %s (uint8, int32 or float32)" % t)


def _acc_code(t: torch.dtype) -> int:
    if t == torch.int32:
        return FHT_I32
    if t == torch.float32:
        return FHT_F32
    raise ValueError("Hough dtype must be int32 or float32")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_2d(x: torch.Tensor, name: str, shape=None, dtype=None):
    """The C entry points see only pointers and pitches, so the extent every
    kernel reads or writes is checked here: 2-D, unit column stride, a row
    pitch covering a row, and (when given) the exact shape and dtype.  The
    device is checked last, so a mis-shaped tensor is reported as such."""
    if x.dim() != 2 or x.stride(1) != 1 or (x.shape[0] > 1 and x.stride(0) < x.shape[1]):
        raise ValueError("%s must be 2-D with unit column stride and a row pitch >= its width" % name)
    if shape is not None and tuple(x.shape) != tuple(int(v) for v in shape):
        raise ValueError("%s must be %dx%d, got %dx%d" % (name, shape[0], shape[1], x.shape[0], x.shape[1]))
    if dtype is not None and x.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, x.dtype))


def _check_device(**tensors):
    """Last check before a call into the library: every tensor on a GPU."""
    for name, x in tensors.items():
        if not x.is_cuda:
            raise ValueError("%s must be a device tensor" % name)


def _check_workspace(ws: torch.Tensor, need: int, name: str = "workspace"):
    if ws.dtype != torch.uint8 or ws.dim() != 1 or not ws.is_contiguous():
        raise ValueError("%s must be a contiguous 1-D uint8 tensor" % name)
    if ws.numel() < need:
        raise ValueError("%s holds %d bytes, %d needed" % (name, ws.numel(), need))
    if ws.data_ptr() % 256:
        raise ValueError("%s must be 256-byte aligned" % name)


def _workspace(nbytes: int, device) -> torch.Tensor:
    # 256-byte aligned by the caching allocator
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def hough_shape(w: int, h: int, quads="full"):
    r, c = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fht_hough_shape(w, h, _quads(quads), ctypes.byref(r), ctypes.byref(c)), "fht_hough_shape")
    return r.value, c.value


def range_shape(w: int, h: int, S1: int, S: int, transposed: bool = False):
    r, c = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fht_range_shape(w, h, S1, S, int(transposed), ctypes.byref(r), ctypes.byref(c)),
           "fht_range_shape")
    return r.value, c.value


def pass_split(side: int):
    n = ctypes.c_int()
    arr = (ctypes.c_int * 4)()
    _check(lib().fht_pass_split(side, ctypes.byref(n), arr), "fht_pass_split")
    return [arr[i] for i in range(n.value)]


def set_pass_split(k: int, passes=None):
    """Stage split for quadrants of 2^k rows (None restores the default);
    calls and batch plans created from now on use it."""
    if passes is None:
        _check(lib().fht_set_pass_split(k, 0, None), "fht_set_pass_split")
        return
    arr = (ctypes.c_int * len(passes))(*passes)
    _check(lib().fht_set_pass_split(k, len(passes), arr), "fht_set_pass_split")


def set_tile_rows(k: int, rows: int | None = None):
    """Tile height (32 or 64) for passes of at most 5 stages of quadrants
    with 2^k rows (None restores the default rule); calls and batch plans
    created from now on use it."""
    _check(lib().fht_set_tile_rows(k, 0 if rows is None else int(rows)), "fht_set_tile_rows")


def tile_rows(side: int) -> int:
    r = ctypes.c_int()
    _check(lib().fht_tile_rows(side, ctypes.byref(r)), "fht_tile_rows")
    return r.value


def autotune(w: int, h: int, in_dtype=torch.float32, reps: int = 20):
    """Time every candidate stage split for an h x w full transform on the
    current device and keep the fastest (fht_autotune); returns the splits
    now used for both sides."""
    it, at, _ = _dtypes(in_dtype)
    _check(lib().fht_autotune(w, h, it, at, reps, _stream()), "fht_autotune")
    return pass_split(h), pass_split(w)


def workspace_size(w: int, h: int, quads="full", in_dtype=torch.float32) -> int:
    it, at, _ = _dtypes(in_dtype)
    b = ctypes.c_size_t()
    _check(lib().fht_workspace_size(w, h, _quads(quads), it, at, ctypes.byref(b)), "fht_workspace_size")
    return b.value


def forward(img: torch.Tensor, quads="full", shifted: bool = False, out: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None, op: str = "sum") -> torch.Tensor:
    """Hough image of a 2-D device image (uint8 -> int32, int32, float32).
    op="max" takes the maximum along every pattern instead of the sum
    (section 1: any associative, commutative operation)."""
    if op not in ("sum", "max"):
        raise ValueError("op must be 'sum' or 'max'")
    _check_2d(img, "img")
    h, w = img.shape
    it, at, odt = _dtypes(img.dtype)
    q = _quads(quads)
    rows, cols = hough_shape(w, h, q)
    if out is None:
        out = torch.empty((rows, cols), dtype=odt, device=img.device)
    _check_2d(out, "out", (rows, cols), odt)
    nb = workspace_size(w, h, q, img.dtype)
    if workspace is None:
        workspace = _workspace(nb, img.device)
    _check_workspace(workspace, nb)
    flags = (FHT_FLAG_SHIFTED if shifted else 0) | (FHT_FLAG_MAX if op == "max" else 0)
    _check_device(img=img, out=out, workspace=workspace)
    rc = lib().fht_forward(img.data_ptr(), it, w, h, img.stride(0), out.data_ptr(), at, out.stride(0), q,
                           flags, workspace.data_ptr(),
                           workspace.numel() * workspace.element_size(), _stream())
    _check(rc, "fht_forward")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # FHT_NOALLOC_SCRATCH_BYTES


def forward_noalloc(img: torch.Tensor, out: torch.Tensor, quads="full", shifted: bool = False,
                    op: str = "sum") -> torch.Tensor:
    """forward() through fht_forward_noalloc: no workspace, the library's own
    per-device scratch array (transforms needing more than
    NOALLOC_SCRATCH_BYTES raise ValueError).  The caller passes `out`; calls
    that overlap in time on one GPU race on the shared scratch."""
    if op not in ("sum", "max"):
        raise ValueError("op must be 'sum' or 'max'")
    _check_2d(img, "img")
    h, w = img.shape
    it, at, odt = _dtypes(img.dtype)
    q = _quads(quads)
    rows, cols = hough_shape(w, h, q)
    _check_2d(out, "out", (rows, cols), odt)
    flags = (FHT_FLAG_SHIFTED if shifted else 0) | (FHT_FLAG_MAX if op == "max" else 0)
    _check_device(img=img, out=out)
    rc = lib().fht_forward_noalloc(img.data_ptr(), it, w, h, img.stride(0), out.data_ptr(), at, out.stride(0), q,
                                   flags, _stream())
    _check(rc, "fht_forward_noalloc")
    return out


def engine_status(workspace: torch.Tensor):
    """Raises FHTError (FHT_ERR_TIMEOUT) if the last call run by the opt-in
    persistent engine (FHT_ENGINE=1) on this workspace had a dependency wait
    give up; waits for the current stream."""
    _check_device(workspace=workspace)
    _check(lib().fht_engine_status(workspace.data_ptr(), _stream()), "fht_engine_status")


def range_params(n: int, deg_lo: float, deg_hi: float):
    """Integer range (S1, S) covering inclinations [deg_lo, deg_hi] (degrees
    from the vertical, positive = leaning right as y grows) for n pattern rows:
    shifts 0..S hold slopes (s - S1)/(n-1)."""
    if n <= 1:
        return 0, 0
    lo = (n - 1) * math.tan(math.radians(deg_lo))
    hi = (n - 1) * math.tan(math.radians(deg_hi))
    S1 = -math.floor(lo)
    S = math.ceil(hi) - math.floor(lo)
    return int(S1), int(S)


def range_workspace_size(w: int, h: int, S1: int, S: int, transposed: bool = False,
                         in_dtype=torch.float32) -> int:
    it, at, _ = _dtypes(in_dtype)
    b = ctypes.c_size_t()
    _check(lib().fht_range_workspace_size(w, h, S1, S, int(transposed), it, at, ctypes.byref(b)),
           "fht_range_workspace_size")
    return b.value


def range_transform(img: torch.Tensor, S1: int, S: int, transposed: bool = False,
                    out: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Angle-range transform (section 4): (S+1) x W."""
    _check_2d(img, "img")
    h, w = img.shape
    it, at, odt = _dtypes(img.dtype)
    rows, cols = range_shape(w, h, S1, S, transposed)
    if out is None:
        out = torch.empty((rows, cols), dtype=odt, device=img.device)
    _check_2d(out, "out", (rows, cols), odt)
    need = range_workspace_size(w, h, S1, S, transposed, img.dtype)
    ws = _workspace(need, img.device) if workspace is None else workspace
    _check_workspace(ws, need)
    _check_device(img=img, out=out, workspace=ws)
    rc = lib().fht_range(img.data_ptr(), it, w, h, img.stride(0), S1, S, int(transposed), out.data_ptr(), at,
                         out.stride(0), ws.data_ptr(), ws.numel(), _stream())
    _check(rc, "fht_range")
    return out


def range_scaled_shape(w: int, h: int, num: int, den: int, S1: int, S: int, transposed: bool = False):
    r, c = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fht_range_scaled_shape(w, h, num, den, S1, S, int(transposed), ctypes.byref(r), ctypes.byref(c)),
           "fht_range_scaled_shape")
    return r.value, c.value


def range_scaled_workspace_size(w: int, h: int, num: int, den: int, S1: int, S: int, transposed: bool = False,
                                in_dtype=torch.float32) -> int:
    it, at, _ = _dtypes(in_dtype)
    b = ctypes.c_size_t()
    _check(lib().fht_range_scaled_workspace_size(w, h, num, den, S1, S, int(transposed), it, at, ctypes.byref(b)),
           "fht_range_scaled_workspace_size")
    return b.value


def range_scaled(img: torch.Tensor, num: int, den: int, S1: int, S: int, transposed: bool = False,
                 out: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Angle range (section 4) of the image scaled by num/den along the
    sheared axis, nearest source sample (see include/fht.h)."""
    _check_2d(img, "img")
    h, w = img.shape
    it, at, odt = _dtypes(img.dtype)
    rows, cols = range_scaled_shape(w, h, num, den, S1, S, transposed)
    if out is None:
        out = torch.empty((rows, cols), dtype=odt, device=img.device)
    _check_2d(out, "out", (rows, cols), odt)
    need = range_scaled_workspace_size(w, h, num, den, S1, S, transposed, img.dtype)
    ws = _workspace(need, img.device) if workspace is None else workspace
    _check_workspace(ws, need)
    _check_device(img=img, out=out, workspace=ws)
    rc = lib().fht_range_scaled(img.data_ptr(), it, w, h, img.stride(0), num, den, S1, S, int(transposed),
                                out.data_ptr(), at, out.stride(0), ws.data_ptr(), ws.numel(), _stream())
    _check(rc, "fht_range_scaled")
    return out


def range_adjoint_workspace_size(w: int, h: int, S1: int, S: int, transposed: bool = False,
                                 dtype=torch.float32) -> int:
    b = ctypes.c_size_t()
    _check(lib().fht_range_adjoint_workspace_size(w, h, S1, S, int(transposed), _acc_code(dtype), ctypes.byref(b)),
           "fht_range_adjoint_workspace_size")
    return b.value


def range_adjoint(grad: torch.Tensor, w: int, h: int, S1: int, S: int, transposed: bool = False,
                  out: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Adjoint of range_transform: (S+1) x W gradient -> h x w image gradient."""
    t = _acc_code(grad.dtype)
    rows, cols = range_shape(w, h, S1, S, transposed)
    _check_2d(grad, "grad", (rows, cols))
    if out is None:
        out = torch.empty((h, w), dtype=grad.dtype, device=grad.device)
    _check_2d(out, "out", (h, w), grad.dtype)
    need = range_adjoint_workspace_size(w, h, S1, S, transposed, grad.dtype)
    ws = _workspace(need, grad.device) if workspace is None else workspace
    _check_workspace(ws, need)
    _check_device(grad=grad, out=out, workspace=ws)
    rc = lib().fht_range_adjoint(grad.data_ptr(), t, grad.stride(0), S1, S, int(transposed), out.data_ptr(),
                                 out.stride(0), w, h, ws.data_ptr(), ws.numel(), _stream())
    _check(rc, "fht_range_adjoint")
    return out


class RangeFunction(torch.autograd.Function):
    """Differentiable angle-range transform of a float32 image (section 4)."""

    @staticmethod
    def forward(ctx, img, S1, S, transposed=False):
        ctx.shape = tuple(img.shape)
        ctx.args = (int(S1), int(S), bool(transposed))
        return range_transform(img.contiguous(), S1, S, transposed)

    @staticmethod
    def backward(ctx, g):
        h, w = ctx.shape
        S1, S, tr = ctx.args
        return range_adjoint(g.contiguous(), w, h, S1, S, tr), None, None, None


def range_pieces(h: int, w: int, deg_lo: float, deg_hi: float):
    """Split an inclination range [deg_lo, deg_hi] (degrees from the vertical,
    -90 <= deg_lo <= deg_hi <= 90, positive = x grows with y) into range
    calls (section 4).  Mostly vertical inclinations |phi| <= 45 run on the
    image; mostly horizontal ones on the transposed image, where a line of
    inclination phi has inclination 90 - phi (phi > 45) or -90 - phi
    (phi < -45).  In each family the integer slope steps k = (n-1) tan(phi)
    from floor to ceil are cut into chunks of at most n steps (one call
    computes shifts 0..S <= n-1); chunk [k0, k1] is S1 = -k0, S = k1 - k0, and
    its row s holds slope (s + k0) / (n - 1).  Returns a list of dicts with
    keys transposed, n, S1, S, k (= (k0, k1))."""
    if not (-90.0 <= deg_lo <= deg_hi <= 90.0):
        raise ValueError("need -90 <= deg_lo <= deg_hi <= 90")
    pieces = []

    def family(lo, hi, transposed):
        n = 1 << max(0, (int(w if transposed else h) - 1).bit_length())
        if n == 1:
            pieces.append(dict(transposed=transposed, n=1, S1=0, S=0, k=(0, 0)))
            return
        k0 = math.floor((n - 1) * math.tan(math.radians(lo)) + 1e-9)
        k1 = math.ceil((n - 1) * math.tan(math.radians(hi)) - 1e-9)
        k0, k1 = max(k0, -(n - 1)), min(k1, n - 1)
        a = k0
        while a <= k1:
            b = min(a + n - 1, k1)
            pieces.append(dict(transposed=transposed, n=n, S1=-a, S=b - a, k=(a, b)))
            a = b + 1

    if deg_hi >= -45.0 and deg_lo <= 45.0:
        family(max(deg_lo, -45.0), min(deg_hi, 45.0), False)
    if deg_hi > 45.0:
        family(90.0 - deg_hi, 90.0 - max(deg_lo, 45.0), True)
    if deg_lo < -45.0:
        family(-90.0 - min(deg_hi, -45.0), -90.0 - deg_lo, True)
    return pieces


def range_any(img: torch.Tensor, deg_lo: float, deg_hi: float):
    """Angle-range transforms covering [deg_lo, deg_hi]: a list of
    (piece, Hough image) with the pieces of range_pieces."""
    h, w = img.shape
    return [(p, range_transform(img, p["S1"], p["S"], p["transposed"])) for p in range_pieces(h, w, deg_lo, deg_hi)]


def range_degrees(img: torch.Tensor, deg_lo: float, deg_hi: float, transposed: bool = False):
    h, w = img.shape
    n = 1 << max(0, (int(w if transposed else h) - 1).bit_length())
    S1, S = range_params(n, deg_lo, deg_hi)
    return range_transform(img, S1, S, transposed), (S1, S)


def shift(hough: torch.Tensor, w: int, h: int, inverse: bool = False, out: torch.Tensor | None = None):
    """fhtshift (section 5) of a full Hough image; out=hough rolls in place."""
    t = _acc_code(hough.dtype)
    rows, cols = hough_shape(w, h)
    _check_2d(hough, "hough", (rows, cols))
    if out is None:
        out = torch.empty_like(hough)
    _check_2d(out, "out", (rows, cols), hough.dtype)
    _check_device(hough=hough, out=out)
    rc = lib().fht_shift(hough.data_ptr(), hough.stride(0), out.data_ptr(), out.stride(0), t, w, h,
                         int(inverse), _stream())
    _check(rc, "fht_shift")
    return out


def adjoint_workspace_size(w: int, h: int, quads="full", dtype=torch.float32) -> int:
    b = ctypes.c_size_t()
    _check(lib().fht_adjoint_workspace_size(w, h, _quads(quads), _acc_code(dtype), ctypes.byref(b)),
           "fht_adjoint_workspace_size")
    return b.value


def adjoint(grad: torch.Tensor, w: int, h: int, quads="full", shifted: bool = False,
            out: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Transpose of forward: Hough-shaped gradient -> h x w image gradient."""
    t = _acc_code(grad.dtype)
    q = _quads(quads)
    _check_2d(grad, "grad", hough_shape(w, h, q))
    if out is None:
        out = torch.empty((h, w), dtype=grad.dtype, device=grad.device)
    _check_2d(out, "out", (h, w), grad.dtype)
    need = adjoint_workspace_size(w, h, q, grad.dtype)
    if workspace is None:
        workspace = _workspace(need, grad.device)
    _check_workspace(workspace, need)
    _check_device(grad=grad, out=out, workspace=workspace)
    rc = lib().fht_adjoint(grad.data_ptr(), t, grad.stride(0), out.data_ptr(), out.stride(0), w, h, q,
                           FHT_FLAG_SHIFTED if shifted else 0, workspace.data_ptr(),
                           workspace.numel() * workspace.element_size(), _stream())
    _check(rc, "fht_adjoint")
    return out


class FHTFunction(torch.autograd.Function):
    """Differentiable full (or partial) Hough transform of float32 images.

    forward: H = F(img) by the library's forward kernels; backward: the
    gradient w.r.t. img is F^T(dL/dH) by the library's adjoint kernels.
    Accepts (h, w) or (batch, h, w).
    """

    @staticmethod
    def forward(ctx, img, quads="full", shifted=False):
        if img.dtype != torch.float32:
            raise ValueError("FHTFunction works on float32 images")
        ctx.quads, ctx.shifted = quads, shifted
        ctx.hw = tuple(img.shape[-2:])
        x = img.contiguous()
        if x.dim() == 2:
            return forward(x, quads, shifted)
        return batch_forward(x, quads, shifted)

    @staticmethod
    def backward(ctx, g):
        h, w = ctx.hw
        g = g.contiguous()
        if g.dim() == 2:
            return adjoint(g, w, h, ctx.quads, ctx.shifted), None, None
        return batch_adjoint(g, w, h, ctx.quads, ctx.shifted, streams=BACKWARD_STREAMS), None, None


# side streams for the backward of an image stack (1: the caller's stream).
# One adjoint launch per pass kind already covers the whole stack, so side
# streams add host work and no overlap (16 x 1024^2: 325 us on one stream,
# 327 us on two).
BACKWARD_STREAMS = 1


def forward_stack_workspace_size(w: int, h: int, n: int, quads="full", in_dtype=torch.float32) -> int:
    it, at, _ = _dtypes(in_dtype)
    b = ctypes.c_size_t()
    _check(lib().fht_forward_stack_workspace_size(w, h, _quads(quads), it, at, n, ctypes.byref(b)),
           "fht_forward_stack_workspace_size")
    return b.value


def batch_forward(x: torch.Tensor, quads="full", shifted: bool = False, out: torch.Tensor | None = None,
                  workspace: torch.Tensor | None = None, op: str = "sum") -> torch.Tensor:
    """Hough images of a (batch, h, w) stack of same-size images, into one
    (batch, rows, cols) tensor (fht_forward_stack: one launch per pass kind
    over the stack, in groups whose bands fit 8 GiB)."""
    if op not in ("sum", "max"):
        raise ValueError("op must be 'sum' or 'max'")
    if x.dim() != 3:
        raise ValueError("batch_forward takes a (batch, h, w) tensor")
    if x.stride(2) != 1 or x.stride(1) < x.shape[2] or x.stride(0) < x.shape[1] * x.stride(1):
        x = x.contiguous()
    n, h, w = x.shape
    it, at, odt = _dtypes(x.dtype)
    q = _quads(quads)
    rows, cols = hough_shape(w, h, q)
    if out is None:
        out = torch.empty((n, rows, cols), dtype=odt, device=x.device)
    elif (out.dim() != 3 or tuple(out.shape) != (n, rows, cols) or out.dtype != odt or out.stride(2) != 1
          or (rows > 1 and out.stride(1) < cols) or (n > 1 and out.stride(0) < rows * out.stride(1))):
        raise ValueError("out must be a (%d, %d, %d) %s tensor with unit column stride" % (n, rows, cols, odt))
    if n == 0:
        return out
    need = forward_stack_workspace_size(w, h, n, q, x.dtype)
    if workspace is None:
        workspace = _workspace(need, x.device)
    _check_workspace(workspace, need)
    flags = (FHT_FLAG_SHIFTED if shifted else 0) | (FHT_FLAG_MAX if op == "max" else 0)
    _check_device(x=x, out=out, workspace=workspace)
    rc = lib().fht_forward_stack(x.data_ptr(), it, w, h, max(x.stride(1), w), x.stride(0), n, out.data_ptr(), at,
                                 max(out.stride(1), cols), out.stride(0), q, flags, workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), _stream())
    _check(rc, "fht_forward_stack")
    return out


def adjoint_stack_workspace_size(w: int, h: int, n: int, quads="full", dtype=torch.float32) -> int:
    b = ctypes.c_size_t()
    _check(lib().fht_adjoint_stack_workspace_size(w, h, _quads(quads), _acc_code(dtype), n, ctypes.byref(b)),
           "fht_adjoint_stack_workspace_size")
    return b.value


_side_streams = {}
_side_workspaces = {}  # (device, streams, index) -> workspace used only on that side stream


def batch_adjoint(g: torch.Tensor, w: int, h: int, quads="full", shifted: bool = False,
                  out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                  streams: int = 1) -> torch.Tensor:
    """Adjoints of a (batch, rows, cols) stack of Hough gradients into one
    (batch, h, w) tensor (fht_adjoint_stack: one launch per pass kind over a
    group of images whose bands fit 2 GiB).  streams > 1 splits the stack into that many parts run
    on side streams of default priority, each with its own workspace (a
    given workspace is then not used); the caller's stream waits for them.
    Inside a stream capture the stack runs on the capturing stream with a
    workspace of its own, so a captured graph never holds a block that later
    eager calls reuse or release."""
    q = _quads(quads)
    rows, cols = hough_shape(w, h, q)
    t = _acc_code(g.dtype)
    if g.dim() != 3 or tuple(g.shape[1:]) != (rows, cols):
        raise ValueError("g must be a (batch, %d, %d) tensor" % (rows, cols))
    n = g.shape[0]
    if out is not None and (out.dim() != 3 or tuple(out.shape) != (n, h, w) or out.dtype != g.dtype
                            or out.stride(2) != 1 or (h > 1 and out.stride(1) < w)
                            or (n > 1 and out.stride(0) < h * out.stride(1))):
        raise ValueError("out must be a (%d, %d, %d) %s tensor with unit column stride" % (n, h, w, g.dtype))
    if not g.is_cuda:
        raise ValueError("g must be a device tensor")
    capturing = torch.cuda.is_current_stream_capturing()
    if streams > 1 and n >= 2 * streams and not capturing:
        if out is None:
            out = torch.empty((n, h, w), dtype=g.dtype, device=g.device)
        cur = torch.cuda.current_stream(g.device)
        key = (g.device, streams)
        if key not in _side_streams:
            _side_streams[key] = [torch.cuda.Stream(device=g.device) for _ in range(streams)]
        side = _side_streams[key]
        bounds = [n * k // streams for k in range(streams + 1)]
        for s in side:
            s.wait_stream(cur)
        for k, s in enumerate(side):
            lo, hi = bounds[k], bounds[k + 1]
            # one workspace per side stream, kept between calls: work on one
            # stream runs in order, so reusing it is safe; a replaced block
            # was allocated on that stream, so the allocator hands it out
            # again only to later work of the same stream
            need = adjoint_stack_workspace_size(w, h, hi - lo, quads, g.dtype)
            wkey = (g.device, streams, k)
            ws = _side_workspaces.get(wkey)
            if ws is None or ws.numel() < need:
                with torch.cuda.stream(s):
                    ws = _workspace(need, g.device)
                _side_workspaces[wkey] = ws
            with torch.cuda.stream(s):
                batch_adjoint(g[lo:hi], w, h, quads, shifted, out=out[lo:hi], workspace=ws)
        for s in side:
            cur.wait_stream(s)
            g.record_stream(s)
            out.record_stream(s)
        return out
    if g.stride(2) != 1 or g.stride(1) < g.shape[2] or g.stride(0) < g.shape[1] * g.stride(1):
        g = g.contiguous()
    if out is None:
        out = torch.empty((n, h, w), dtype=g.dtype, device=g.device)
    if n == 0:
        return out
    need = adjoint_stack_workspace_size(w, h, n, q, g.dtype)
    if workspace is None:
        workspace = _workspace(need, g.device)
    _check_workspace(workspace, need)
    _check_device(g=g, out=out, workspace=workspace)
    rc = lib().fht_adjoint_stack(g.data_ptr(), t, g.stride(1), g.stride(0), out.data_ptr(), out.stride(1),
                                 out.stride(0), w, h, n, q, FHT_FLAG_SHIFTED if shifted else 0,
                                 workspace.data_ptr(), workspace.numel(), _stream())
    _check(rc, "fht_adjoint_stack")
    return out


def fht(img, quads="full", shifted=False):
    return FHTFunction.apply(img, quads, shifted)


def cell_segment(w: int, h: int, row: int, x0: int, quads="full", shifted: bool = False):
    """Image segment of Hough cell (row, x0) (sections 3.2, 3.3): ((xa, ya),
    (xb, yb), pixels) or None in the black zone."""
    seg = (ctypes.c_int32 * 5)()
    _check(lib().fht_cell_segment(w, h, _quads(quads), row, x0, int(shifted), seg), "fht_cell_segment")
    if seg[4] == 0:
        return None
    return (seg[0], seg[1]), (seg[2], seg[3]), seg[4]


def peaks(hough: torch.Tensor, radius: int = 4, threshold: float = 0.0, max_out: int | None = None):
    """Local maxima of a Hough image: [(value, row, col)] by decreasing value
    (ties by index), and the total number found.  With max_out given, at most
    that many (an arbitrary subset when more exist); with None, all of them
    (a second launch when the first buffer was too small)."""
    _check_2d(hough, "hough")
    t = _acc_code(hough.dtype)
    _check_device(hough=hough)
    rows, cols = hough.shape
    cap = max_out if max_out is not None else 65536
    while True:
        out = torch.empty(cap, dtype=torch.int64, device=hough.device)
        count = torch.zeros(1, dtype=torch.int32, device=hough.device)
        _check(lib().fht_peaks(hough.data_ptr(), t, rows, cols, hough.stride(0), radius, float(threshold),
                               out.data_ptr(), cap, count.data_ptr(), _stream()), "fht_peaks")
        total = int(count.item())
        if max_out is not None or total <= cap:
            break
        cap = total
    idx = out[:min(total, cap)]
    res = []
    if idx.numel():
        rr, cc = idx // cols, idx % cols
        vals = hough[rr, cc].cpu().tolist()
        res = sorted(zip(vals, rr.cpu().tolist(), cc.cpu().tolist()), key=lambda e: (-e[0], e[1], e[2]))
    return res, total


def detect_lines(img: torch.Tensor, k: int = 8, radius: int = 4, threshold: float = 0.0):
    """Full forward, the k strongest local maxima, and their image segments:
    [(value, row, x0, segment)] (segment as in cell_segment)."""
    h, w = img.shape
    H = forward(img)
    found, _ = peaks(H, radius, threshold)
    return [(v, r, c, cell_segment(w, h, r, c)) for v, r, c in found[:k]]


def timing_enable(on: bool = True):
    """Start (clearing earlier records) or stop recording HIP events around
    every pass kernel launch of the library."""
    _check(lib().fht_timing_enable(int(on)), "fht_timing_enable")


def timing_filter(substr=None):
    """Record only the kernels whose name contains substr (None: all)."""
    _check(lib().fht_timing_filter(substr.encode() if substr else None), "fht_timing_filter")


def timing_report():
    """{kernel name: (launches, total ms)} of the launches recorded since
    timing_enable(True); waits for the recorded events."""
    L = lib()
    out = {}
    i = 0
    buf = ctypes.create_string_buffer(256)
    while True:
        n, ms = ctypes.c_int64(), ctypes.c_double()
        rc = L.fht_timing_report(i, buf, 256, ctypes.byref(n), ctypes.byref(ms))
        if rc == FHT_ERR_INVALID:
            break
        _check(rc, "fht_timing_report")
        out[buf.value.decode()] = (n.value, ms.value)
        i += 1
    return out


class BatchPlan:
    """Plan for transforming many images of different sizes together: one
    launch per (pass, stages, last-pass) class over every image."""

    def __init__(self, sizes, quads="full", in_dtype=torch.uint8, device=None):
        self.sizes = [(int(h), int(w)) for h, w in sizes]
        self.n = len(self.sizes)
        self.quads = _quads(quads)
        it, at, self.out_dtype = _dtypes(in_dtype)
        self.in_code, self.acc_code = it, at
        self.in_dtype = in_dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        ws = (ctypes.c_int32 * self.n)(*[w for h, w in self.sizes])
        hs = (ctypes.c_int32 * self.n)(*[h for h, w in self.sizes])
        plan = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        tot = ctypes.c_int64()
        offs = (ctypes.c_int64 * self.n)()
        with torch.cuda.device(self.device):
            _check(lib().fht_batch_plan_create(ws, hs, self.n, self.quads, it, at, ctypes.byref(plan),
                                               ctypes.byref(wsb), ctypes.byref(tot), offs),
                   "fht_batch_plan_create")
        self._plan = plan
        self.workspace_bytes = wsb.value
        self.out_elems = tot.value
        self.offsets = [offs[i] for i in range(self.n)]
        self.shapes = [hough_shape(w, h, self.quads) for h, w in self.sizes]
        self._workspace = None

    def output(self) -> torch.Tensor:
        return torch.empty(self.out_elems, dtype=self.out_dtype, device=self.device)

    def views(self, packed: torch.Tensor):
        return [packed[o:o + r * c].view(r, c) for o, (r, c) in zip(self.offsets, self.shapes)]

    def pointer_table(self, imgs) -> torch.Tensor:
        imgs = list(imgs)
        if len(imgs) != self.n:
            raise ValueError("the plan holds %d images, %d given" % (self.n, len(imgs)))
        for x, (h, w) in zip(imgs, self.sizes):
            if x.shape != (h, w) or x.dtype != self.in_dtype or not x.is_contiguous() or x.device != self.device:
                raise ValueError("batch image does not match the plan")
        return torch.tensor([x.data_ptr() for x in imgs], dtype=torch.int64, device=self.device)

    @property
    def workspace(self) -> torch.Tensor:
        """The plan's own workspace (allocated on first use)."""
        if self._workspace is None:
            self._workspace = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        return self._workspace

    def run(self, ptr_table: torch.Tensor, packed: torch.Tensor, workspace: torch.Tensor | None = None):
        """One batched forward on the current stream.  A workspace passed in
        (at least workspace_bytes, 256-byte aligned) is used instead of the
        plan's own, so calls on different streams do not share one."""
        if (ptr_table.dtype != torch.int64 or ptr_table.dim() != 1 or ptr_table.numel() != self.n
                or not ptr_table.is_contiguous()):
            raise ValueError("ptr_table must be a contiguous int64 tensor of %d pointers" % self.n)
        if (packed.dtype != self.out_dtype or not packed.is_contiguous() or packed.numel() < self.out_elems):
            raise ValueError("packed must be a contiguous %s tensor of at least %d elements"
                             % (self.out_dtype, self.out_elems))
        if ptr_table.device != self.device or packed.device != self.device:
            raise ValueError("ptr_table and packed must be on the plan's device")
        ws = self.workspace if workspace is None else workspace
        _check_workspace(ws, self.workspace_bytes, "batch workspace")
        _check_device(ptr_table=ptr_table, packed=packed, workspace=ws)
        rc = lib().fht_batch_forward(self._plan, ptr_table.data_ptr(), packed.data_ptr(), ws.data_ptr(), ws.numel(),
                                     _stream())
        _check(rc, "fht_batch_forward")
        return packed

    def run_stack(self, x: torch.Tensor, packed: torch.Tensor, workspace: torch.Tensor | None = None):
        """One batched forward of a contiguous (n, h, w) stack on the current
        stream, for a plan of n equal sizes: the images' addresses are worked
        out on the device (fht_batch_forward_stack), so no pointer table is
        copied from the host."""
        n = self.n
        if x.dim() != 3 or x.shape[0] != n or not x.is_contiguous() or x.dtype != self.in_dtype:
            raise ValueError("x must be a contiguous (%d, h, w) %s tensor" % (n, self.in_dtype))
        if any(s != (x.shape[1], x.shape[2]) for s in self.sizes):
            raise ValueError("the plan's image sizes do not match the stack")
        if packed.dtype != self.out_dtype or not packed.is_contiguous() or packed.numel() < self.out_elems:
            raise ValueError("packed must be a contiguous %s tensor of at least %d elements"
                             % (self.out_dtype, self.out_elems))
        if x.device != self.device or packed.device != self.device:
            raise ValueError("x and packed must be on the plan's device")
        ws = self.workspace if workspace is None else workspace
        _check_workspace(ws, self.workspace_bytes, "batch workspace")
        _check_device(x=x, packed=packed, workspace=ws)
        rc = lib().fht_batch_forward_stack(self._plan, x.data_ptr(), x.stride(0) * x.element_size(),
                                           packed.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
        _check(rc, "fht_batch_forward_stack")
        return packed

    def __call__(self, imgs):
        packed = self.output()
        self.run(self.pointer_table(imgs), packed)
        return self.views(packed)

    def capture(self, ptr_table: torch.Tensor, packed: torch.Tensor):
        """Capture one batched forward into a HIP graph (torch.cuda.CUDAGraph);
        replaying it reruns the whole batch with the same buffers."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run(ptr_table, packed)  # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(g):
            self.run(ptr_table, packed)
        return g

    def __del__(self):
        p = getattr(self, "_plan", None)
        if p is not None and p.value and _lib is not None:
            _lib.fht_batch_plan_destroy(p)
            self._plan = None
