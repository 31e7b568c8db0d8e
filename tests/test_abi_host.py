"""Host-side tests of the C ABI (no kernel launches): exports, layout, validation."""
import ctypes
import os
import re

import pytest

from oracle import geometry as geo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ct.h")


@pytest.fixture(scope="module")
def ct():
    from paper_1510_00561_amd import ct as ctmod
    if not os.path.exists(ctmod.LIB_PATH):
        from paper_1510_00561_amd import build
        build.build()
    return ctmod


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ct_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(ct):
    lib = ct._lib()
    names = declared_functions()
    assert "ct_forward" in names and "ct_quantize" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in ct.h but not exported"


GEOMS = [
    (256, 256, 2, [8, 4]),
    (480, 640, 3, [16, 8, 4]),
    (1080, 1920, 4, [32, 16, 8, 8]),
    (720, 1280, 3, [16, 8, 4]),
    (240, 320, 4, [16, 8, 8, 8]),
    (70, 90, 3, [16, 8, 4]),
    (128, 128, 1, [64]),
    (64, 96, 2, [4, 32]),
]


@pytest.mark.parametrize("H,W,J,dirs", GEOMS)
def test_layout_matches_oracle(ct, H, W, J, dirs):
    lay, table = ct.layout(H, W, J, dirs)
    ref = geo.subband_table(H, W, J, dirs)
    R, C = geo.padded_size(H, W, J, dirs)
    assert (lay.pad_h, lay.pad_w) == (R, C)
    assert lay.exp2 == geo.pad_exponent(J, dirs)
    assert lay.ncoef == geo.ncoef(H, W, J, dirs)
    assert lay.nsub == len(ref)
    for got, want in zip(table, ref):
        assert (got.level, got.k, got.rows, got.cols, got.offset) == \
               (want.level, want.k, want.rows, want.cols, want.offset)
        assert (got.o1, got.o2, got.s1, got.s2, bool(got.transposed)) == \
               (want.o1, want.o2, want.s1, want.s2, want.transposed)


@pytest.mark.parametrize("H,W,J,dirs", [
    (256, 256, 0, []),
    (256, 256, 7, [4] * 6),
    (256, 256, 2, [8, 6]),
    (256, 256, 2, [128, 4]),
    (256, 256, 2, [2, 4]),
    (8, 256, 2, [32, 4]),
    (0, 256, 1, [4]),
])
def test_layout_rejects_bad_geometry(ct, H, W, J, dirs):
    g = ct.geom(H, W, J, dirs[:6])
    lay = ct.Layout()
    assert ct._lib().ct_layout_query(ctypes.byref(g), ctypes.byref(lay), None, 0) == -2


def test_null_arguments(ct):
    lib = ct._lib()
    g = ct.geom(256, 256, 2, [8, 4])
    assert lib.ct_layout_query(None, None, None, 0) == -1
    assert lib.ct_layout_query(ctypes.byref(g), None, None, 0) == -1
    n = ctypes.c_size_t(7)
    assert lib.ct_workspace_bytes(ctypes.byref(g), -1, ctypes.byref(n)) == -1 and n.value == 0
    dummy = ctypes.c_void_p(0x1000)
    # validation fails before any launch
    assert lib.ct_forward(ctypes.byref(g), 1, None, dummy, dummy, 1 << 40, None) == -1
    assert lib.ct_inverse(ctypes.byref(g), 1, dummy, None, dummy, 1 << 40, None) == -1
    assert lib.ct_forward(ctypes.byref(g), -3, dummy, dummy, dummy, 1 << 40, None) == -1
    assert lib.ct_quantize(ctypes.byref(g), 1, dummy, None, 0, dummy, dummy, dummy, 1 << 40, None) == -1
    assert lib.ct_dequantize(ctypes.byref(g), 1, dummy, dummy, 3, dummy, dummy, None) == -1  # stride < nsub
    assert lib.ct_forward(ctypes.byref(g), 0, None, None, None, 0, None) == 0   # empty batch


def test_workspace_too_small(ct):
    lib = ct._lib()
    g = ct.geom(256, 256, 2, [8, 4])
    need = ct.workspace_bytes(256, 256, 2, [8, 4], 3)
    assert need >= 3 * 256 * 256 * 4 * 3
    dummy = ctypes.c_void_p(0x1000)
    for fn in ("ct_forward", "ct_inverse", "ct_forward_adjoint", "ct_inverse_adjoint"):
        assert getattr(lib, fn)(ctypes.byref(g), 3, dummy, dummy, dummy, need - 1, None) == -3
    assert lib.ct_quantize(ctypes.byref(g), 3, dummy, dummy, 0, dummy, dummy, dummy, need - 1, None) == -3


def test_fault_injection_hook(ct, monkeypatch):
    lib = ct._lib()
    g = ct.geom(256, 256, 2, [8, 4])
    need = ct.workspace_bytes(256, 256, 2, [8, 4], 1)
    dummy = ctypes.c_void_p(0x1000)
    monkeypatch.setenv("CT_FAULT_INJECT", "launch")
    assert lib.ct_forward(ctypes.byref(g), 1, dummy, dummy, dummy, need, None) == -4
    assert lib.ct_quantize(ctypes.byref(g), 1, dummy, dummy, 0, dummy, dummy, dummy, need, None) == -4
    assert lib.ct_rgb_to_ycocg(1, 4, 4, 2, dummy, dummy, dummy, dummy, None) == -4
    assert lib.ct_ycocg_to_rgb(1, 4, 4, 2, dummy, dummy, dummy, dummy, None) == -4
    assert lib.ct_lowpass_diff(ctypes.byref(g), 1, dummy, 1, None) == -4
    assert lib.ct_motion_search(1, 16, 16, 8, dummy, dummy, dummy, None, None) == -4
    other = ctypes.c_void_p(0x2000)
    assert lib.ct_mc_residual(ctypes.byref(g), 1, 1, dummy, dummy, dummy, 16, 16, 1, 0, other, None) == -4
    n = ctypes.c_size_t(0)
    assert lib.ct_rle_workspace_bytes(ctypes.byref(g), 1, ctypes.byref(n)) == 0
    assert lib.ct_rle_encode(ctypes.byref(g), 1, dummy, 0, dummy, dummy, dummy, n.value, None) == -4
    assert lib.ct_strerror(-4) == b"HIP runtime error"


def test_plan_validation_errors(ct):
    lib = ct._lib()
    handle = ctypes.c_void_p()
    assert lib.ct_plan_create(None, 1, 0, ctypes.byref(handle)) == -1
    descs = (ct.StreamDesc * 1)()
    assert lib.ct_plan_create(descs, 0, 0, ctypes.byref(handle)) == -1
    assert lib.ct_plan_create(descs, 1, 0, None) == -1
    d = descs[0]
    d.geom = ct.geom(256, 256, 2, [8, 4])
    d.batch = 1
    dummy = 0x1000
    d.planes = d.coeffs = d.idx = d.side = d.steps = d.deq = d.out = dummy
    d.steps_stride = 3                         # shorter than nsub
    assert lib.ct_plan_create(descs, 1, 0, ctypes.byref(handle)) == -1
    d.steps_stride = 0
    d.out = None
    assert lib.ct_plan_create(descs, 1, 0, ctypes.byref(handle)) == -1
    d.out = dummy
    d.geom = ct.geom(256, 256, 2, [8, 6])      # not a power of two
    assert lib.ct_plan_create(descs, 1, 0, ctypes.byref(handle)) == -2
    d.geom = ct.geom(256, 256, 2, [8, 4])
    d.batch = 0
    assert lib.ct_plan_create(descs, 1, 0, ctypes.byref(handle)) == -1
    assert handle.value is None
    assert lib.ct_plan_run(None, None) == -1
    assert lib.ct_plan_run_plain(None, None) == -1
    info = ct.PlanInfo()
    assert lib.ct_plan_info(None, ctypes.byref(info)) == -1
    lib.ct_plan_destroy(None)


def test_colour_and_lowpass_validation(ct):
    # every error path returns before any launch, so this runs without a GPU
    lib = ct._lib()
    d4 = ctypes.c_void_p(0x1000)       # 16-byte aligned dummies
    odd = ctypes.c_void_p(0x1004)      # 4-byte but not 16-byte aligned
    for fn in ("ct_rgb_to_ycocg", "ct_ycocg_to_rgb"):
        f = getattr(lib, fn)
        assert f(0, 4, 4, 2, None, None, None, None, None) == 0          # empty batch
        assert f(1, 4, 4, 0, d4, d4, d4, d4, None) == -1                 # n < 1
        assert f(1, 4, 4, 65, d4, d4, d4, d4, None) == -1                # n > maximum
        assert f(-1, 4, 4, 1, d4, d4, d4, d4, None) == -1
        assert f(1, 0, 4, 1, d4, d4, d4, d4, None) == -1
        assert f(1, 4, 4, 1, d4, d4, None, d4, None) == -1               # null plane
        assert f(1 << 10, 1 << 10, 1 << 10, 1, d4, d4, d4, d4, None) == -1   # 2^31 elements
    assert lib.ct_rgb_to_ycocg(1, 4, 4, 1, d4, odd, d4, d4, None) == -1  # Y not 16-byte aligned
    assert lib.ct_rgb_to_ycocg(1, 4, 4, 1, ctypes.c_void_p(0x1002), d4, d4, d4, None) == -1
    assert lib.ct_ycocg_to_rgb(1, 4, 4, 1, d4, d4, d4, odd, None) == -1  # RGB not 16-byte aligned
    g = ct.geom(256, 256, 2, [8, 4])
    assert lib.ct_lowpass_diff(None, 1, d4, 0, None) == -1
    assert lib.ct_lowpass_diff(ctypes.byref(g), 1, None, 0, None) == -1
    assert lib.ct_lowpass_diff(ctypes.byref(g), -1, d4, 0, None) == -1
    assert lib.ct_lowpass_diff(ctypes.byref(g), 0, None, 0, None) == 0
    bad = ct.geom(256, 256, 2, [8, 6])
    assert lib.ct_lowpass_diff(ctypes.byref(bad), 1, d4, 0, None) == -2


def test_motion_search_validation(ct):
    lib = ct._lib()
    d = ctypes.c_void_p(0x1000)
    f = lib.ct_motion_search
    assert f(0, 16, 16, 8, None, None, None, None, None) == 0     # empty batch
    assert f(1, 16, 16, 0, d, d, d, d, None) == -1                # w < 1
    assert f(1, 16, 16, 17, d, d, d, d, None) == -1               # w > 16
    assert f(1, 0, 16, 8, d, d, d, d, None) == -1
    assert f(-1, 16, 16, 8, d, d, d, d, None) == -1
    assert f(1, 16, 16, 8, None, d, d, d, None) == -1
    assert f(1, 16, 16, 8, d, d, None, d, None) == -1
    assert f(1 << 12, 1 << 10, 1 << 10, 8, d, d, d, d, None) == -1   # 2^32 pixels


def test_quantize_noalloc_validation(ct):
    # every check runs before the first HIP call, so this runs without a GPU
    lib = ct._lib()
    g = ct.geom(256, 256, 2, [8, 4])
    d = ctypes.c_void_p(0x1000)
    f = lib.ct_quantize_noalloc
    assert f(ctypes.byref(g), 0, None, None, 0, None, None, None) == 0    # empty batch
    assert f(None, 1, d, d, 0, d, d, None) == -1
    assert f(ctypes.byref(g), -1, d, d, 0, d, d, None) == -1
    assert f(ctypes.byref(g), 1, None, d, 0, d, d, None) == -1
    assert f(ctypes.byref(g), 1, d, d, 3, d, d, None) == -1              # stride < nsub
    assert f(ctypes.byref(g), 1025, d, d, 0, d, d, None) == -3           # beyond the static scratch
    bad = ct.geom(256, 256, 2, [8, 6])
    assert f(ctypes.byref(bad), 1, d, d, 0, d, d, None) == -2


def test_variant_fields_validated(ct):
    """ct_geom.filters and .recon: 0 and 1 are served, anything else is a
    geometry error; the layout does not depend on them."""
    lib = ct._lib()
    n = ctypes.c_size_t(0)
    base = ct.layout(70, 90, 3, [16, 8, 4])[0]
    for f, r in ((0, 0), (1, 0), (0, 1), (1, 1)):
        g = ct.geom(70, 90, 3, [16, 8, 4], f, r)
        assert lib.ct_workspace_bytes(ctypes.byref(g), 2, ctypes.byref(n)) == 0
        lay = ct.Layout()
        assert lib.ct_layout_query(ctypes.byref(g), ctypes.byref(lay), None, 0) == 0
        assert (lay.pad_h, lay.pad_w, lay.ncoef, lay.nsub) == (base.pad_h, base.pad_w, base.ncoef, base.nsub)
    assert ct.geom(70, 90, 3, [16, 8, 4], "53", "ba").filters == 1
    assert ct.geom(70, 90, 3, [16, 8, 4], "53", "ba").recon == 1
    for f, r in ((2, 0), (-1, 0), (0, 2), (0, -1)):
        g = ct.geom(70, 90, 3, [16, 8, 4], f, r)
        assert lib.ct_workspace_bytes(ctypes.byref(g), 2, ctypes.byref(n)) == -2
        d = ctypes.c_void_p(0x1000)
        assert lib.ct_forward(ctypes.byref(g), 1, d, d, d, 1 << 30, None) == -2


def test_autotune_validation(ct):
    """ct_autotune checks its arguments before any HIP call."""
    lib = ct._lib()
    g = ct.geom(256, 256, 2, [32, 4])
    d = ctypes.c_void_p(0x1000)
    n = ctypes.c_size_t(0)
    assert lib.ct_workspace_bytes(ctypes.byref(g), 2, ctypes.byref(n)) == 0
    assert lib.ct_autotune(None, 1, d, n.value, None) == -1
    assert lib.ct_autotune(ctypes.byref(g), -1, d, n.value, None) == -1
    assert lib.ct_autotune(ctypes.byref(g), 0, None, 0, None) == 0          # empty batch
    assert lib.ct_autotune(ctypes.byref(g), 2, None, n.value, None) == -1
    assert lib.ct_autotune(ctypes.byref(g), 2, d, n.value - 1, None) == -3
    bad = ct.geom(256, 256, 2, [32, 6])
    assert lib.ct_autotune(ctypes.byref(bad), 2, d, n.value, None) == -2
    assert lib.ct_autotune_clear() == 0


def test_encode_rgb_validation(ct):
    """ct_encode_rgb checks its arguments before any launch: the frame count
    (negative, or 3 * frames past the batch limit), null pointers, the steps
    stride, the workspace size for 3 * frames planes; zero frames is a no-op."""
    lib = ct._lib()
    g = ct.geom(256, 256, 2, [8, 4])
    dummy = ctypes.c_void_p(0x1000)
    need = ct.workspace_bytes(256, 256, 2, [8, 4], 6)
    assert lib.ct_encode_rgb(ctypes.byref(g), -1, dummy, dummy, 0, dummy, dummy, dummy, need, None) == -1
    assert lib.ct_encode_rgb(ctypes.byref(g), 21846, dummy, dummy, 0, dummy, dummy, dummy, 1 << 50, None) == -1
    assert lib.ct_encode_rgb(ctypes.byref(g), 2, None, dummy, 0, dummy, dummy, dummy, need, None) == -1
    assert lib.ct_encode_rgb(ctypes.byref(g), 2, dummy, dummy, 3, dummy, dummy, dummy, need, None) == -1
    assert lib.ct_encode_rgb(ctypes.byref(g), 2, dummy, dummy, 0, dummy, dummy, dummy, need - 1, None) == -3
    assert lib.ct_encode_rgb(ctypes.byref(g), 0, None, None, 0, None, None, None, 0, None) == 0
    bad = ct.geom(256, 256, 2, [8, 4], filters="53")
    bad.filters = 7
    assert lib.ct_encode_rgb(ctypes.byref(bad), 1, dummy, dummy, 0, dummy, dummy, dummy, 1 << 40, None) == -2
