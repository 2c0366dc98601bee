"""ctypes wrapper around fht_oracle.c (test infrastructure only).

Every array crossing into C is float64, C-contiguous.  Integer images are
exact in float64 as long as every partial sum stays below 2**53, which the
wrappers assert.  Each function names the paper section it follows; the C
source carries the details.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fht_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_D = ctypes.c_double
_I64 = ctypes.c_int64
_PD = ctypes.POINTER(ctypes.c_double)


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over rows)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            lib = ctypes.CDLL(_LIB)
            lib.oracle_threads.restype = ctypes.c_int
            lib.oracle_threads.argtypes = []
            lib.oracle_next_pow2.restype = _I64
            lib.oracle_next_pow2.argtypes = [_I64]
            lib.oracle_pattern_offset.restype = _I64
            lib.oracle_pattern_offset.argtypes = [_I64, _I64, _I64]
            lib.oracle_quadrant.restype = ctypes.c_int
            lib.oracle_quadrant.argtypes = [_PD, _I64, _I64, _I64, ctypes.c_int, ctypes.c_int, _PD]
            lib.oracle_full.restype = ctypes.c_int
            lib.oracle_full.argtypes = [_PD, _I64, _I64, _I64, ctypes.c_int, _PD]
            lib.oracle_range_adjoint.restype = ctypes.c_int
            lib.oracle_range_adjoint.argtypes = [_PD, _I64, _I64, _I64, _I64, ctypes.c_int, ctypes.c_int, _PD,
                                                 _I64]
            lib.oracle_range_scaled.restype = ctypes.c_int
            lib.oracle_range_scaled.argtypes = [_PD, _I64, _I64, _I64, _I64, _I64, _I64, _I64, ctypes.c_int,
                                                ctypes.c_int, _PD]
            lib.oracle_quadrant_op.restype = ctypes.c_int
            lib.oracle_quadrant_op.argtypes = [_PD, _I64, _I64, _I64, ctypes.c_int, ctypes.c_int, _PD]
            lib.oracle_full_op.restype = ctypes.c_int
            lib.oracle_full_op.argtypes = [_PD, _I64, _I64, _I64, ctypes.c_int, _PD]
            lib.oracle_row_quadrant.restype = ctypes.c_int
            lib.oracle_row_quadrant.argtypes = [_I64, _I64, _I64, ctypes.POINTER(_I64)]
            lib.oracle_fhtshift_roll.restype = _I64
            lib.oracle_fhtshift_roll.argtypes = [ctypes.c_int, _I64, _I64, _I64]
            lib.oracle_fhtshift_full.restype = ctypes.c_int
            lib.oracle_fhtshift_full.argtypes = [_PD, _I64, _I64, ctypes.c_int, _PD]
            lib.oracle_range_sigma.restype = _I64
            lib.oracle_range_sigma.argtypes = [_I64, _I64, _I64]
            lib.oracle_range.restype = ctypes.c_int
            lib.oracle_range.argtypes = [_PD, _I64, _I64, _I64, _I64, _I64, ctypes.c_int,
                                         ctypes.c_int, _PD]
            lib.oracle_cell.restype = _D
            lib.oracle_cell.argtypes = [_PD, _I64, _I64, _I64, ctypes.c_int, _I64, _I64]
            lib.oracle_full_cell.restype = _D
            lib.oracle_full_cell.argtypes = [_PD, _I64, _I64, _I64, _I64, _I64]
            lib.oracle_adjoint_full.restype = ctypes.c_int
            lib.oracle_adjoint_full.argtypes = [_PD, _I64, _I64, ctypes.c_int, _PD, _I64]
            lib.oracle_adjoint_quadrant.restype = ctypes.c_int
            lib.oracle_adjoint_quadrant.argtypes = [_PD, _I64, _I64, ctypes.c_int, ctypes.c_int,
                                                    _PD, _I64]
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def _as_f64(img) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(img), dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("image must be 2-D (h, w)")
    return a


def _check_exact(img: np.ndarray, n_terms: int):
    # integer data stays exact in float64 while every partial sum is < 2**53
    if np.all(np.isfinite(img)) and np.all(img == np.round(img)):
        bound = float(np.max(np.abs(img))) * n_terms if img.size else 0.0
        if bound >= 2.0 ** 53:
            raise ValueError("integer sums would exceed float64's exact range")


def _rc(rc: int):
    if rc == -1:
        raise ValueError("oracle: bad argument")
    if rc == -2:
        raise MemoryError("oracle: out of memory")
    if rc != 0:
        raise RuntimeError("oracle: status %d" % rc)


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(_load().oracle_threads())


def next_pow2(v: int) -> int:
    return int(_load().oracle_next_pow2(int(v)))


def pattern_offset(n: int, s: int, y: int) -> int:
    """D_n(s, y), Brady's dyadic pattern (section 2)."""
    return int(_load().oracle_pattern_offset(n, s, y))


def hough_shape(w: int, h: int):
    hp, wp = next_pow2(h), next_pow2(w)
    return 2 * (hp + wp) - 3, hp + wp


def quadrant(img, q: int, single: bool = False) -> np.ndarray:
    """One quadrant (section 3.1), n x W by the stage recurrence."""
    a = _as_f64(img)
    h, w = a.shape
    hp, wp = next_pow2(h), next_pow2(w)
    n = hp if q <= 2 else wp
    _check_exact(a, max(hp, wp))
    out = np.empty((n, hp + wp), dtype=np.float64)
    _rc(_load().oracle_quadrant(_ptr(a), w, h, w, q, int(single), _ptr(out)))
    return out


def stacked_quadrants(img, quads, single: bool = False) -> np.ndarray:
    """Unmerged quadrants in increasing order, stacked along rows."""
    return np.concatenate([quadrant(img, q, single) for q in sorted(quads)], axis=0)


def full(img, single: bool = False) -> np.ndarray:
    """Full Hough image (section 3.3), (2(w'+h')-3) x W."""
    a = _as_f64(img)
    h, w = a.shape
    rows, W = hough_shape(w, h)
    _check_exact(a, max(next_pow2(h), next_pow2(w)))
    out = np.empty((rows, W), dtype=np.float64)
    _rc(_load().oracle_full(_ptr(a), w, h, w, int(single), _ptr(out)))
    return out


def range_adjoint(g, w: int, h: int, S1: int, S: int, transposed: bool = False, single: bool = False) -> np.ndarray:
    """Adjoint of range_transform (section 4): (S+1) x W gradient -> h x w."""
    a = _as_f64(g)
    out = np.empty((h, w), dtype=np.float64)
    _rc(_load().oracle_range_adjoint(_ptr(a), w, h, S1, S, int(transposed), int(single), _ptr(out), w))
    return out


def scaled_sizes(w: int, h: int, num: int, den: int, transposed: bool = False):
    """Image sizes after scaling the sheared axis by num/den (ceil)."""
    if transposed:
        return w, -(-h * num // den)
    return -(-w * num // den), h


def range_scaled(img, num: int, den: int, S1: int, S: int, transposed: bool = False,
                 single: bool = False) -> np.ndarray:
    """Angle range of the image scaled by num/den along the sheared axis
    (section 4), nearest-sample reading: (S+1) x W of the scaled sizes."""
    a = _as_f64(img)
    h, w = a.shape
    ws, hs = scaled_sizes(w, h, num, den, transposed)
    W = next_pow2(ws) + next_pow2(hs)
    out = np.empty((S + 1, W), dtype=np.float64)
    _rc(_load().oracle_range_scaled(_ptr(a), w, h, w, num, den, S1, S, int(transposed), int(single), _ptr(out)))
    return out


_OPS = {"sum": 0, "max": 1}


def quadrant_op(img, q: int, op: str = "sum") -> np.ndarray:
    """One quadrant with `op` along the patterns (section 1: any associative,
    commutative operation; "max" here)."""
    a = _as_f64(img)
    h, w = a.shape
    hp, wp = next_pow2(h), next_pow2(w)
    n = hp if q <= 2 else wp
    out = np.empty((n, hp + wp), dtype=np.float64)
    _rc(_load().oracle_quadrant_op(_ptr(a), w, h, w, q, _OPS[op], _ptr(out)))
    return out


def full_op(img, op: str = "sum") -> np.ndarray:
    """Full Hough image (section 3.3 layout) with `op` along the patterns."""
    a = _as_f64(img)
    h, w = a.shape
    rows, W = hough_shape(w, h)
    out = np.empty((rows, W), dtype=np.float64)
    _rc(_load().oracle_full_op(_ptr(a), w, h, w, _OPS[op], _ptr(out)))
    return out


def row_quadrant(w: int, h: int, r: int):
    """(quadrant, local shift) of full-image row r (section 3.3)."""
    s = _I64(0)
    q = _load().oracle_row_quadrant(w, h, r, ctypes.byref(s))
    return int(q), int(s.value)


def fhtshift_roll(q: int, hp: int, wp: int, s: int) -> int:
    return int(_load().oracle_fhtshift_roll(q, hp, wp, s))


def fhtshift_full(hough, w: int, h: int, inverse: bool = False) -> np.ndarray:
    """fhtshift (section 5) of a full Hough image."""
    a = np.ascontiguousarray(hough, dtype=np.float64)
    rows, W = hough_shape(w, h)
    if a.shape != (rows, W):
        raise ValueError("shape mismatch")
    out = np.empty_like(a)
    _rc(_load().oracle_fhtshift_full(_ptr(a), w, h, int(inverse), _ptr(out)))
    return out


def range_sigma(n: int, S1: int, y: int) -> int:
    return int(_load().oracle_range_sigma(n, S1, y))


def range_params(n: int, deg_lo: float, deg_hi: float):
    """Integer range (S1, S) for inclinations [deg_lo, deg_hi] in degrees.

    Inclination = deviation of the line from the vertical axis; slope
    dx/dy = tan(angle).  Shifts 0..S cover slopes (s - S1)/(n - 1).
    """
    if n <= 1:
        return 0, 0
    lo = (n - 1) * math.tan(math.radians(deg_lo))
    hi = (n - 1) * math.tan(math.radians(deg_hi))
    S1 = -math.floor(lo)
    S = math.ceil(hi) - math.floor(lo)
    return int(S1), int(S)


def range_transform(img, S1: int, S: int, transposed: bool = False,
                    single: bool = False) -> np.ndarray:
    """Angle-range variant (section 4): (S+1) x W."""
    a = _as_f64(img)
    h, w = a.shape
    hp, wp = next_pow2(h), next_pow2(w)
    _check_exact(a, max(hp, wp))
    out = np.empty((S + 1, hp + wp), dtype=np.float64)
    _rc(_load().oracle_range(_ptr(a), w, h, w, S1, S, int(transposed), int(single), _ptr(out)))
    return out


def cell(img, q: int, s: int, x: int) -> float:
    """One quadrant cell by its definition (sum along one pattern)."""
    a = _as_f64(img)
    h, w = a.shape
    return float(_load().oracle_cell(_ptr(a), w, h, w, q, s, x))


def full_cell(img, r: int, x: int, _cache=None) -> float:
    a = _as_f64(img)
    h, w = a.shape
    return float(_load().oracle_full_cell(_ptr(a), w, h, w, r, x))


def full_cells(img, rows, cols) -> np.ndarray:
    """Many full-image cells by definition (for sampled checks at full size)."""
    a = _as_f64(img)
    h, w = a.shape
    lib = _load()
    p = _ptr(a)
    return np.array([lib.oracle_full_cell(p, w, h, w, int(r), int(x)) for r, x in zip(rows, cols)],
                    dtype=np.float64)


def adjoint_full(grad, w: int, h: int, single: bool = False) -> np.ndarray:
    """Transpose of the full Hough transform: (rows x W) -> h x w."""
    g = np.ascontiguousarray(grad, dtype=np.float64)
    rows, W = hough_shape(w, h)
    if g.shape != (rows, W):
        raise ValueError("shape mismatch")
    out = np.empty((h, w), dtype=np.float64)
    _rc(_load().oracle_adjoint_full(_ptr(g), w, h, int(single), _ptr(out), w))
    return out


def adjoint_quadrant(grad, w: int, h: int, q: int, single: bool = False) -> np.ndarray:
    g = np.ascontiguousarray(grad, dtype=np.float64)
    hp, wp = next_pow2(h), next_pow2(w)
    n = hp if q <= 2 else wp
    if g.shape != (n, hp + wp):
        raise ValueError("shape mismatch")
    out = np.empty((h, w), dtype=np.float64)
    _rc(_load().oracle_adjoint_quadrant(_ptr(g), w, h, q, int(single), _ptr(out), w))
    return out
