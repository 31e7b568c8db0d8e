"""Pins of the oracle's contourlet-domain motion compensation (paper section
3.7): hand-worked vector mapping, zero vectors, a global shift of a periodic
frame (which the transform's shift covariance turns into shifted components,
so the prediction must reproduce the current frame's coefficients), the
padding rows, and the exact decoder round trip."""
import json
import os

import numpy as np
import pytest

from oracle import ct as oct
from oracle import geometry as geo
from oracle import mc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mc_worked.json")


def _random_idx(table, seed, lo=-300, hi=300):
    n = table[-1].offset + table[-1].size
    return np.random.default_rng(seed).integers(lo, hi, size=n).astype(np.int16)


def test_worked_vector_mapping():
    g = json.load(open(GOLDEN))
    H, W, J, dirs = g["geometry"]
    table = geo.subband_table(H, W, J, dirs)
    dy, dx = g["vector"]
    nby, nbx = -(-H // 16), -(-W // 16)
    mv = np.tile(np.array([dy, dx]), (nby, nbx, 1))
    for c in g["cases"]:
        sb = next(s for s in table if s.level == c["level"] and (s.cone == c["cone"] or c["cone"] == "L" and s.k < 0))
        assert mc.spacing(sb, J, c["n"]) == tuple(c["spacing"])
        di, dk = mc.component_vectors(sb, J, mv, c["n"])
        assert np.all(di == c["mapped"][0]) and np.all(dk == c["mapped"][1]), c


def test_round_div_halves_away_from_zero():
    assert list(mc.round_div([5, -5, 3, -3, 1, -1, 0, 7], 2)) == [3, -3, 2, -2, 1, -1, 0, 4]
    assert list(mc.round_div([6, -6, 2, -2, 10], 4)) == [2, -2, 1, -1, 3]


@pytest.mark.parametrize("H,W,J,dirs", [(64, 96, 2, [8, 4]), (70, 90, 3, [16, 8, 4]), (64, 96, 2, [4, 32])])
def test_zero_vectors_give_plain_differences(H, W, J, dirs):
    table = geo.subband_table(H, W, J, dirs)
    cur, prev = _random_idx(table, 1), _random_idx(table, 2)
    mv = np.zeros((-(-H // 16), -(-W // 16), 2), np.int64)
    want = (cur.astype(np.int64) - prev).astype(np.int16)
    np.testing.assert_array_equal(mc.residual_plane(cur, prev, table, J, mv), want)


@pytest.mark.parametrize("H,W,J,dirs,shift", [
    (64, 96, 2, [8, 4], (8, -12)),
    (64, 96, 2, [4, 32], (-32, 64)),     # e = 5: shifts by multiples of 32 map exactly
    (128, 128, 1, [64], (32, -64)),
])
def test_global_shift_is_predicted_exactly(H, W, J, dirs, shift):
    # cur[y][x] = prev[y + dy][x + dx] on the torus: every block's vector is
    # (dy, dx), and by shift covariance every component of cur is the
    # previous component displaced by the mapped vector
    R, C = geo.padded_size(H, W, J, dirs)
    assert (R, C) == (H, W)
    e = geo.pad_exponent(J, dirs)
    dy, dx = shift
    assert dy % (1 << e) == 0 and dx % (1 << e) == 0 and dy != dx
    x = np.random.default_rng(5).uniform(0, 255, (H, W))
    prev = oct.forward(x, J, dirs)
    cur = oct.forward(np.roll(x, (-dy, -dx), axis=(0, 1)), J, dirs)
    table = geo.subband_table(H, W, J, dirs)
    mv = np.tile(np.array([dy, dx]), (H // 16, W // 16, 1))
    pred = mc.predict_plane(prev, table, J, mv)
    assert np.abs(pred - cur).max() < 1e-9
    # transposing the vector (or reading a transposed subband in its stored
    # orientation) does not predict it
    bad = mc.predict_plane(prev, table, J, mv[..., ::-1])
    assert np.abs(bad - cur).max() > 1.0


def test_padding_rows_take_the_last_block():
    # 70 x 90 pads to 72 x 96: samples in the padding belong to the last
    # block row / column, whose vector is the only non-zero one
    H, W, J, dirs = 70, 90, 3, [16, 8, 4]
    table = geo.subband_table(H, W, J, dirs)
    nby, nbx = -(-H // 16), -(-W // 16)
    mv = np.zeros((nby, nbx, 2), np.int64)
    mv[-1, -1] = (32, 32)
    for sb in table:
        di, dk = mc.component_vectors(sb, J, mv)
        py, px = mc.sample_pixels(sb, J)
        moved = (di != 0) | (dk != 0)
        inside = (py >= 16 * (nby - 1)) & (px >= 16 * (nbx - 1))
        assert not np.any(moved & ~inside)
        sy, sx = mc.spacing(sb, J)
        if 32 * 2 >= sy and 32 * 2 >= sx:     # the mapped vector is non-zero
            assert np.all(moved[inside])


@pytest.mark.parametrize("n", [1, 2])
def test_decoder_restores_exactly(n):
    H, W, J, dirs = 70, 90, 3, [16, 8, 4]
    table = geo.subband_table(H, W, J, dirs)
    cur, prev = _random_idx(table, 3, -32768, 32767), _random_idx(table, 4, -32768, 32767)
    rng = np.random.default_rng(9)
    mv = rng.integers(-8, 9, size=(-(-H // 16), -(-W // 16), 2))
    r = mc.residual_plane(cur, prev, table, J, mv, n)
    assert r.dtype == np.int16
    np.testing.assert_array_equal(mc.restore_plane(r, prev, table, J, mv, n), cur)
