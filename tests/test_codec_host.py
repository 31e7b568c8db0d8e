"""Host code of the codec back end (no GPU): the library's run-length decoder
and its DEFLATE / INFLATE (paper sections 3.8, 3.9) against the oracle's
symbol streams and zlib byte counts."""
import ctypes

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import rle


@pytest.fixture(scope="module")
def ct():
    import os
    from paper_1510_00561_amd import ct as ctmod
    if not os.path.exists(ctmod.LIB_PATH):
        from paper_1510_00561_amd import build
        build.build()
    return ctmod


GEOMS = [(16, 16, 1, [4]), (64, 96, 2, [4, 32]), (70, 90, 3, [16, 8, 4]), (40, 40, 3, [8, 4, 4])]


def _plane(table, density, seed):
    rng = np.random.default_rng(seed)
    n = table[-1].offset + table[-1].size
    return np.where(rng.random(n) < density, rng.integers(-300, 301, n), 0).astype(np.int16)


@pytest.mark.parametrize("H,W,J,dirs", GEOMS)
@pytest.mark.parametrize("p_frame", [0, 1])
def test_host_decoder_inverts_oracle_streams(ct, H, W, J, dirs, p_frame):
    table = geo.subband_table(H, W, J, dirs)
    plan = ct.Plan.__new__(ct.Plan)          # host-only use: geometry and layout, no workspace
    plan.g = ct.geom(H, W, J, dirs)
    plan.ncoef = table[-1].offset + table[-1].size
    for density in (0.0, 0.03, 0.4, 1.0):
        idx = _plane(table, density, H + int(100 * density))
        sym, off = rle.encode_plane(idx, table, p_frame)
        np.testing.assert_array_equal(plan.rle_decode_host(sym, off.astype(np.int32), p_frame), idx)


def test_host_decoder_rejects_bad_streams(ct):
    H, W, J, dirs = 16, 16, 1, [4]
    table = geo.subband_table(H, W, J, dirs)
    idx = _plane(table, 0.2, 1)
    sym, off = rle.encode_plane(idx, table, 1)
    g = ct.geom(H, W, J, dirs)
    out = np.empty(len(idx), np.int16)
    lib = ct._lib()
    off32 = off.astype(np.int32)
    bad = sym.copy()
    z = int(np.flatnonzero(bad == 0)[0])
    bad[z + 1] = 10000                       # a run past the end of its row
    assert lib.ct_rle_decode_host(ctypes.byref(g), bad.ctypes.data, off32.ctypes.data, 1, out.ctypes.data) == -1
    short = off32.copy()
    short[-1] -= 1                           # the last component ends early
    assert lib.ct_rle_decode_host(ctypes.byref(g), sym.ctypes.data, short.ctypes.data, 1, out.ctypes.data) == -1
    assert lib.ct_rle_decode_host(ctypes.byref(g), None, off32.ctypes.data, 1, out.ctypes.data) == -1


@pytest.mark.parametrize("mode", [0, 1])
def test_deflate_matches_zlib_and_round_trips(ct, mode):
    table = geo.subband_table(64, 96, 2, [4, 32])
    idx = _plane(table, 0.1, 7)
    sym, off = rle.encode_plane(idx, table, 0)
    blob, parts = ct.deflate_host(sym, off.astype(np.int32), mode)
    per, whole = rle.deflate_sizes(sym, off)
    if mode == 0:
        assert list(parts) == per and len(blob) == sum(per)
    else:
        assert list(parts) == [whole] and len(blob) == whole
    np.testing.assert_array_equal(ct.inflate_host(blob, parts, off.astype(np.int32), mode), sym)


def test_codec_validation(ct):
    lib = ct._lib()
    g = ct.geom(64, 96, 2, [4, 32])
    d = ctypes.c_void_p(0x1000)
    assert lib.ct_mc_residual(ctypes.byref(g), 0, 1, None, None, None, 1, 1, 1, 0, None, None) == 0
    assert lib.ct_mc_residual(ctypes.byref(g), 1, 0, d, d, d, 4, 6, 1, 0, ctypes.c_void_p(0x2000), None) == -1
    assert lib.ct_mc_residual(ctypes.byref(g), 1, 1, d, d, d, 0, 6, 1, 0, ctypes.c_void_p(0x2000), None) == -1
    assert lib.ct_mc_residual(ctypes.byref(g), 1, 1, d, d, d, 4, 6, 1, 0, d, None) == -1   # out aliases prev
    assert lib.ct_mc_residual(ctypes.byref(g), 1, 1, None, d, d, 4, 6, 1, 0, ctypes.c_void_p(0x2000), None) == -1
    n = ctypes.c_size_t(0)
    assert lib.ct_rle_workspace_bytes(ctypes.byref(g), 2, ctypes.byref(n)) == 0 and n.value > 0
    assert lib.ct_rle_encode(ctypes.byref(g), 2, d, 0, d, d, d, n.value - 1, None) == -3
    assert lib.ct_rle_encode(ctypes.byref(g), 2, None, 0, d, d, d, n.value, None) == -1
    assert lib.ct_rle_encode(ctypes.byref(g), 0, None, 0, None, None, None, 0, None) == 0
    bad = ct.geom(64, 96, 2, [4, 6])
    assert lib.ct_rle_encode(ctypes.byref(bad), 1, d, 0, d, d, d, 1 << 30, None) == -2
