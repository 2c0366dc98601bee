"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re

import pytest
import torch

from paper_1811_06378_amd import fht

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fht.h")

pytestmark = pytest.mark.skipif(not os.path.exists(fht.LIB_PATH), reason="libfht.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fht_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = _declared()
    assert "fht_forward" in names and "fht_adjoint" in names and "fht_range" in names and "fht_shift" in names
    L = fht.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fht.SIGNATURES), "binding signatures must cover the header exactly"


def test_version_and_strings():
    L = fht.lib()
    assert L.fht_version() >= 10000
    for rc in (0, -1, -2, -3, -4, -5):
        assert L.fht_status_string(rc)


def test_adjoint_stack_sizes_and_validation():
    L = fht.lib()
    one = fht.adjoint_workspace_size(300, 200)
    one256 = (one + 255) // 256 * 256
    assert fht.adjoint_stack_workspace_size(300, 200, 1) == one256
    assert fht.adjoint_stack_workspace_size(300, 200, 3) == 3 * one256
    assert fht.adjoint_stack_workspace_size(300, 200, 100) == 100 * one256  # one group
    # groups keep their bands within 2 GiB: 4096^2 images (275 MB of bands each) run 7 at a time
    big = (fht.adjoint_workspace_size(4096, 4096) + 255) // 256 * 256
    per_group = (2 << 30) // big
    assert 1 <= per_group < 16
    assert fht.adjoint_stack_workspace_size(4096, 4096, 16) == per_group * big
    assert fht.adjoint_stack_workspace_size(4096, 4096, 1) == big
    rows, cols = fht.hough_shape(300, 200)
    p = ctypes.c_void_p(1 << 20)
    args = dict(t=fht.FHT_F32, ld=cols, gs=rows * cols, ldi=300, istr=300 * 200, n=3)

    def call(**kw):
        a = {**args, **kw}
        return L.fht_adjoint_stack(p, a["t"], a["ld"], a["gs"], p, a["ldi"], a["istr"], 300, 200, a["n"], 15, 0,
                                   p, 1 << 40, None)
    assert call(n=0) == fht.FHT_ERR_INVALID
    assert call(gs=rows * cols - 1) == fht.FHT_ERR_INVALID
    assert call(istr=300 * 200 - 1) == fht.FHT_ERR_INVALID
    assert call(t=fht.FHT_U8) == fht.FHT_ERR_INVALID
    assert call(ld=cols - 1) == fht.FHT_ERR_INVALID


def test_forward_stack_sizes_and_validation():
    L = fht.lib()
    one = (fht.workspace_size(300, 200, "full", torch.uint8) + 255) // 256 * 256
    assert fht.forward_stack_workspace_size(300, 200, 1, "full", torch.uint8) == one
    assert fht.forward_stack_workspace_size(300, 200, 50, "full", torch.uint8) == 50 * one
    # groups keep their bands within 8 GiB: 8192^2 float32 images run 3 at a time
    big = (fht.workspace_size(8192, 8192) + 255) // 256 * 256
    per_group = (8 << 30) // big
    assert 1 <= per_group < 8
    assert fht.forward_stack_workspace_size(8192, 8192, 8) == per_group * big
    rows, cols = fht.hough_shape(300, 200)
    p = ctypes.c_void_p(1 << 20)
    args = dict(it=fht.FHT_U8, at=fht.FHT_I32, ldi=300, istr=300 * 200, n=3, ldh=cols, hstr=rows * cols,
                ws=1 << 40, wsp=p, flags=0, q=15)

    def call(**kw):
        a = {**args, **kw}
        return L.fht_forward_stack(p, a["it"], 300, 200, a["ldi"], a["istr"], a["n"], p, a["at"], a["ldh"], a["hstr"],
                                   a["q"], a["flags"], a["wsp"], a["ws"], None)
    assert call(n=0) == fht.FHT_ERR_INVALID
    assert call(istr=300 * 200 - 1) == fht.FHT_ERR_INVALID
    assert call(hstr=rows * cols - 1) == fht.FHT_ERR_INVALID
    assert call(ldi=299) == fht.FHT_ERR_INVALID
    assert call(ldh=cols - 1) == fht.FHT_ERR_INVALID
    assert call(at=fht.FHT_F32) == fht.FHT_ERR_INVALID
    assert call(flags=1, q=1) == fht.FHT_ERR_INVALID  # fhtshift needs the full image
    assert call(ws=3 * one - 1) == fht.FHT_ERR_WORKSPACE
    assert call(wsp=None) == fht.FHT_ERR_WORKSPACE
    assert call(wsp=ctypes.c_void_p((1 << 20) + 64)) == fht.FHT_ERR_INVALID
    assert L.fht_forward_stack(None, fht.FHT_U8, 300, 200, 300, 60000, 3, p, fht.FHT_I32, cols, rows * cols, 15, 0,
                               p, 1 << 40, None) == fht.FHT_ERR_INVALID
    with pytest.raises(ValueError):
        fht.forward_stack_workspace_size(300, 200, 0)


def test_timing_filter_and_empty_report_need_no_gpu():
    # the filter is a host-side string; an empty record set reports nothing
    fht.timing_filter("fht_pass_kernel<float")
    fht.timing_filter("x" * 1000)  # truncated, not an error
    fht.timing_filter(None)
    fht.timing_enable(False)
    assert fht.lib().fht_timing_report(10 ** 6, None, 0, None, None) == fht.FHT_ERR_INVALID


@pytest.mark.parametrize("w,h,quads,rows,cols", [
    (1, 1, 15, 1, 2), (1024, 1024, 15, 4093, 2048), (4096, 4096, 15, 16381, 8192),
    (100, 37, 15, 2 * (128 + 64) - 3, 192), (100, 37, 1, 64, 192), (100, 37, 4, 128, 192),
    (100, 37, 5, 192, 192), (100, 37, 14, 64 + 128 + 128, 192)])
def test_hough_shape(w, h, quads, rows, cols):
    assert fht.hough_shape(w, h, quads) == (rows, cols)


@pytest.mark.parametrize("args", [(0, 5, 15), (5, 0, 15), (5, 5, 0), (5, 5, 16), (70000, 5, 15)])
def test_hough_shape_rejects(args):
    with pytest.raises(ValueError):
        fht.hough_shape(*args)


def test_range_shape():
    assert fht.range_shape(1024, 1024, 275, 550) == (551, 2048)
    with pytest.raises(ValueError):
        fht.range_shape(1024, 1024, 275, 1024)
    with pytest.raises(ValueError):
        fht.range_shape(1024, 1024, -1024, 5)


def test_pass_split():
    assert fht.pass_split(4096) == [6, 6]
    assert fht.pass_split(1024) == [6, 4]
    assert fht.pass_split(512) == [6, 3]
    assert fht.pass_split(256) == [5, 3]
    assert fht.pass_split(128) == [4, 3]
    assert fht.pass_split(2048) == [6, 5]
    assert fht.pass_split(64) == [6]
    assert fht.pass_split(3) == [2]
    assert fht.pass_split(8192) == [5, 4, 4]
    for side in [1, 2, 5, 8, 100, 3000, 65536]:
        k = max(0, (side - 1).bit_length())
        assert sum(fht.pass_split(side)) == k


def test_workspace_size_monotone():
    a = fht.workspace_size(1024, 1024)
    b = fht.workspace_size(4096, 4096)
    assert 0 < a < b
    # one pass: no intermediate band, only the 256-byte queue/counter area
    assert fht.workspace_size(64, 64) == 256


def test_validation_before_hip():
    """Invalid calls return a negative status without any HIP call (works on a
    machine with no GPU)."""
    L = fht.lib()
    s = ctypes.c_void_p(0)
    dummy = ctypes.c_void_p(0x1000)
    # null image
    assert L.fht_forward(None, 2, 8, 8, 8, dummy, 2, 16, 15, 0, None, 0, s) == fht.FHT_ERR_INVALID
    # bad dtype pair
    assert L.fht_forward(dummy, 0, 8, 8, 8, dummy, 2, 16, 15, 0, None, 0, s) == fht.FHT_ERR_INVALID
    # pitch too small
    assert L.fht_forward(dummy, 2, 8, 8, 7, dummy, 2, 16, 15, 0, None, 0, s) == fht.FHT_ERR_INVALID
    assert L.fht_forward(dummy, 2, 8, 8, 8, dummy, 2, 15, 15, 0, None, 0, s) == fht.FHT_ERR_INVALID
    # shifted needs the full image
    assert L.fht_forward(dummy, 2, 8, 8, 8, dummy, 2, 16, 1, 1, None, 0, s) == fht.FHT_ERR_INVALID
    # workspace missing for a two-pass size
    assert L.fht_forward(dummy, 2, 1024, 1024, 1024, dummy, 2, 2048, 15, 0, None, 0, s) == fht.FHT_ERR_WORKSPACE
    assert L.fht_forward(dummy, 2, 1024, 1024, 1024, dummy, 2, 2048, 15, 0, dummy, 16, s) == fht.FHT_ERR_WORKSPACE
    assert b"workspace" in L.fht_last_error()
    # range bounds
    assert L.fht_range(dummy, 0, 64, 64, 64, 0, 64, 0, dummy, 1, 128, None, 0, s) == fht.FHT_ERR_INVALID
    # adjoint type
    assert L.fht_adjoint(dummy, 0, 16, dummy, 8, 8, 8, 15, 0, None, 0, s) == fht.FHT_ERR_INVALID
    # the max transform has no adjoint; unknown flag bits are rejected
    assert L.fht_adjoint(dummy, 2, 16, dummy, 8, 8, 8, 15, fht.FHT_FLAG_MAX, None, 0, s) == fht.FHT_ERR_INVALID
    assert L.fht_forward(dummy, 2, 8, 8, 8, dummy, 2, 16, 15, 4, None, 0, s) == fht.FHT_ERR_INVALID
    # fhtshift overlap that is not identity
    assert L.fht_shift(dummy, 16, ctypes.c_void_p(0x1004), 16, 2, 8, 8, 0, s) == fht.FHT_ERR_INVALID
    # engine status needs the workspace it reads
    assert L.fht_engine_status(None, s) == fht.FHT_ERR_INVALID
    # the allocation-free forward validates like fht_forward, and rejects
    # transforms whose bands exceed its scratch before touching the device
    assert L.fht_forward_noalloc(None, 2, 8, 8, 8, dummy, 2, 16, 15, 0, s) == fht.FHT_ERR_INVALID
    assert L.fht_forward_noalloc(dummy, 2, 8, 8, 7, dummy, 2, 16, 15, 0, s) == fht.FHT_ERR_INVALID
    assert L.fht_forward_noalloc(dummy, 2, 2048, 2048, 2048, dummy, 2, 4096, 15, 0, s) == fht.FHT_ERR_UNSUPPORTED
    assert b"allocation-free" in L.fht_last_error()
    # batch: bad sizes
    p = ctypes.c_void_p()
    wsb, tot = ctypes.c_size_t(), ctypes.c_int64()
    ws = (ctypes.c_int32 * 2)(8, 0)
    hs = (ctypes.c_int32 * 2)(8, 8)
    assert L.fht_batch_plan_create(ws, hs, 2, 15, 0, 1, ctypes.byref(p), ctypes.byref(wsb), ctypes.byref(tot),
                                   None) in (fht.FHT_ERR_INVALID, fht.FHT_ERR_UNSUPPORTED)


def test_range_params_helper():
    assert fht.range_params(1024, -15, 15) == (275, 550)
    assert fht.range_params(1, -15, 15) == (0, 0)


def test_product_path_has_no_oracle_import():
    """The package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_1811_06378_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "fht_oracle" not in text, f


def test_batch_plan_host_side():
    """Plan arguments are validated before any HIP call."""
    L = fht.lib()
    p = ctypes.c_void_p()
    wsb, tot = ctypes.c_size_t(), ctypes.c_int64()
    ws = (ctypes.c_int32 * 2)(0, 8)
    hs = (ctypes.c_int32 * 2)(8, 8)
    assert L.fht_batch_plan_create(ws, hs, 2, 15, 0, 1, ctypes.byref(p), ctypes.byref(wsb), ctypes.byref(tot),
                                   None) == fht.FHT_ERR_INVALID
    ws[0] = 65537
    assert L.fht_batch_plan_create(ws, hs, 2, 15, 0, 1, ctypes.byref(p), ctypes.byref(wsb), ctypes.byref(tot),
                                   None) == fht.FHT_ERR_INVALID
    ws[0] = 3
    assert L.fht_batch_plan_create(ws, hs, 2, 15, 2, 1, ctypes.byref(p), ctypes.byref(wsb), ctypes.byref(tot),
                                   None) == fht.FHT_ERR_INVALID
    assert L.fht_batch_plan_create(ws, hs, 2, 0, 0, 1, ctypes.byref(p), ctypes.byref(wsb), ctypes.byref(tot),
                                   None) == fht.FHT_ERR_INVALID
    assert L.fht_batch_plan_destroy(None) == 0


def test_range_scaled_shape_and_validation():
    L = fht.lib()
    r, c = ctypes.c_int64(), ctypes.c_int64()
    # 100 columns scaled by 3/2 -> 150 -> w' = 256; h' = 64
    assert L.fht_range_scaled_shape(100, 64, 3, 2, 5, 40, 0, ctypes.byref(r), ctypes.byref(c)) == 0
    assert (r.value, c.value) == (41, 256 + 64)
    # transposed: the rows are scaled: 64 -> 32 rows -> h' = 32, n = w' = 128
    assert L.fht_range_scaled_shape(100, 64, 1, 2, 5, 40, 1, ctypes.byref(r), ctypes.byref(c)) == 0
    assert (r.value, c.value) == (41, 128 + 32)
    assert L.fht_range_scaled_shape(100, 64, 0, 2, 5, 40, 0, ctypes.byref(r), ctypes.byref(c)) == fht.FHT_ERR_INVALID
    assert L.fht_range_scaled_shape(100, 64, 65, 1, 5, 40, 0, ctypes.byref(r), ctypes.byref(c)) == fht.FHT_ERR_INVALID


def test_set_pass_split_validation_and_roundtrip():
    try:
        assert fht.pass_split(1024) == [6, 4]
        fht.set_pass_split(10, [4, 6])
        assert fht.pass_split(1024) == [4, 6]
        assert fht.pass_split(2048) == [6, 5]          # other k untouched
        for bad in ([5, 6], [2, 8], [10], [3, 3, 4]):
            with pytest.raises(ValueError):
                fht.set_pass_split(10, bad)
        with pytest.raises(ValueError):
            fht.set_pass_split(2, [2])
        # the first band is other + 2^G1 - 1 columns (origin rounded to 64):
        # a deeper first pass never needs less workspace
        fht.set_pass_split(10, [6, 4])
        wide = fht.workspace_size(1024, 1024)
        fht.set_pass_split(10, [4, 6])
        assert fht.workspace_size(1024, 1024) <= wide
    finally:
        fht.set_pass_split(10, None)
    assert fht.pass_split(1024) == [6, 4]


# The C entry points see only pointers and pitches; the binding checks every
# tensor's extent and dtype first.  CPU tensors suffice: a mis-shaped tensor
# is rejected for its shape (the device check comes last), so no call
# reaches the library's launch path.
def _shape_error(fn, *a, **kw):
    import torch  # noqa: F401
    with pytest.raises(ValueError) as e:
        fn(*a, **kw)
    msg = str(e.value)
    assert "device tensor" not in msg, msg
    return msg


def test_binding_rejects_misshaped_tensors_before_any_launch():
    import torch
    w, h = 30, 20
    rows, cols = fht.hough_shape(w, h)
    img = torch.zeros((h, w), dtype=torch.float32)
    G = torch.zeros((rows, cols), dtype=torch.float32)
    # forward: out of the wrong shape or dtype
    _shape_error(fht.forward, img, out=torch.zeros((rows - 1, cols)))
    _shape_error(fht.forward, img, out=torch.zeros((rows, cols), dtype=torch.int32))
    _shape_error(fht.forward, img, out=torch.zeros((rows, cols)), workspace=torch.zeros(16, dtype=torch.uint8))
    # adjoint: gradient short by a row, image gradient short by a row
    _shape_error(fht.adjoint, torch.zeros((rows - 1, cols)), w, h)
    _shape_error(fht.adjoint, G, w, h, out=torch.zeros((h - 1, w)))
    _shape_error(fht.adjoint, torch.zeros((fht.hough_shape(w, h, [1])[0], cols)), w, h)  # quadrant, not full
    # batch adjoint: per-image gradient shape, output shape
    _shape_error(fht.batch_adjoint, torch.zeros((2, rows, cols - 1)), w, h)
    _shape_error(fht.batch_adjoint, torch.zeros((2, rows, cols)), w, h, out=torch.zeros((2, h, w - 1)))
    # fhtshift: a quadrant-only image, or an output of another shape
    _shape_error(fht.shift, torch.zeros((32, cols)), w, h)
    _shape_error(fht.shift, G, w, h, out=torch.zeros((rows, cols + 1)))
    # angle range, scaled range and range adjoint: outputs and gradients
    S1, S = 3, 9
    rr, rc = fht.range_shape(w, h, S1, S)
    _shape_error(fht.range_transform, img, S1, S, out=torch.zeros((rr + 1, rc)))
    sr, sc = fht.range_scaled_shape(w, h, 2, 1, S1, S)
    _shape_error(fht.range_scaled, img, 2, 1, S1, S, out=torch.zeros((sr, sc - 1)))
    _shape_error(fht.range_adjoint, torch.zeros((rr - 1, rc)), w, h, S1, S)
    _shape_error(fht.range_adjoint, torch.zeros((rr, rc)), w, h, S1, S, out=torch.zeros((h, w + 1)))
    # rows with a pitch below their width
    _shape_error(fht.forward, torch.zeros((h, w)).as_strided((h, w), (w - 1, 1)))
    # correct shapes pass every shape check (a host workspace may then fail
    # the 256-byte alignment check before the device check)
    with pytest.raises(ValueError, match="device tensor|256-byte aligned"):
        fht.forward(img, out=torch.zeros((rows, cols)))
    with pytest.raises(ValueError, match="device tensor|256-byte aligned"):
        fht.adjoint(G, w, h, out=torch.zeros((h, w)))


def test_tile_rows_setting_and_validation():
    """The tile height of passes of at most 5 stages: 32 by default, settable
    per stage count, validated before any HIP call."""
    assert fht.tile_rows(1024) == 32
    fht.set_tile_rows(10, 64)
    try:
        assert fht.tile_rows(1024) == 64
        assert fht.tile_rows(512) == 32
    finally:
        fht.set_tile_rows(10, None)
    assert fht.tile_rows(1024) == 32
    for k, rows in [(2, 32), (17, 32), (10, 48), (10, 16)]:
        with pytest.raises(ValueError):
            fht.set_tile_rows(k, rows)
    with pytest.raises(ValueError):
        fht.tile_rows(0)
