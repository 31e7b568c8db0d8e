"""Pins of the oracle's zero-run coder (paper section 3.8) and DEFLATE stage
(section 3.9): hand-worked rows, the natural (image-row) orientation of
transposed subbands, the symbol count by an independent route, K- and
P-frame component choice, and exact round trips."""
import json
import os
import zlib

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import rle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rle_worked.json")


def test_worked_rows():
    for case in json.load(open(GOLDEN))["rows"]:
        assert rle.rle_row(case["row"]) == case["symbols"]
        row, pos = rle.unrle_row(case["symbols"], 0, len(case["row"]))
        assert row == case["row"] and pos == len(case["symbols"])


def _sparse_plane(table, density, seed):
    rng = np.random.default_rng(seed)
    n = table[-1].offset + table[-1].size
    vals = rng.integers(-40, 41, size=n)
    keep = rng.random(n) < density
    return np.where(keep, vals, 0).astype(np.int16)


def _runs_in_rows(mask2d):
    """Number of maximal True runs along each row, counted from run starts."""
    m = np.asarray(mask2d, dtype=bool)
    starts = m & ~np.concatenate([np.zeros((m.shape[0], 1), bool), m[:, :-1]], axis=1)
    return int(starts.sum())


@pytest.mark.parametrize("H,W,J,dirs", [(16, 16, 1, [4]), (32, 48, 2, [8, 4]), (40, 40, 3, [8, 4, 4]),
                                        (64, 96, 2, [4, 32])])
@pytest.mark.parametrize("p_frame", [False, True])
def test_symbol_count_and_round_trip(H, W, J, dirs, p_frame):
    table = geo.subband_table(H, W, J, dirs)
    for density in (0.0, 0.05, 0.5, 1.0):
        idx = _sparse_plane(table, density, seed=int(density * 100) + H)
        sym, off = rle.encode_plane(idx, table, p_frame)
        assert off[0] == 0 and off[-1] == len(sym)
        for s, sb in enumerate(table):
            comp = idx[sb.offset:sb.offset + sb.size]
            if rle.coded(sb, p_frame):
                nat = comp.reshape(sb.cols, sb.rows).T if sb.transposed else comp.reshape(sb.rows, sb.cols)
                want = int(np.count_nonzero(nat)) + 2 * _runs_in_rows(nat == 0)
            else:
                want = sb.size
                np.testing.assert_array_equal(sym[off[s]:off[s + 1]], comp)
            assert off[s + 1] - off[s] == want, (s, density)
        np.testing.assert_array_equal(rle.decode_plane(sym, off, table, p_frame), idx)


def test_kframe_lowpass_not_coded_pframe_lowpass_coded():
    table = geo.subband_table(32, 48, 2, [8, 4])
    idx = np.zeros(table[-1].offset + table[-1].size, np.int16)
    low = table[0]
    k_sym, k_off = rle.encode_plane(idx, table, False)
    p_sym, p_off = rle.encode_plane(idx, table, True)
    assert k_off[1] == low.size                       # raw lowpass
    assert p_off[1] == 2 * low.rows                   # one run per lowpass row
    assert k_off[-1] - k_off[1] == p_off[-1] - p_off[1]


def test_transposed_subband_is_coded_along_image_rows():
    # one non-zero coefficient at natural (row 1, column 2) of a vertical-cone
    # subband: the runs must be counted along natural rows, i.e. down the
    # stored columns
    table = geo.subband_table(16, 16, 1, [4])
    sb = next(s for s in table if s.transposed)
    idx = np.zeros(table[-1].offset + table[-1].size, np.int16)
    nat = np.zeros((sb.rows, sb.cols), np.int16)
    nat[1, 2] = 9
    idx[sb.offset:sb.offset + sb.size] = nat.T.reshape(-1)
    sym, off = rle.encode_plane(idx, table, True)
    s = table.index(sb)
    got = list(sym[off[s]:off[s + 1]])
    c = sb.cols
    want = [0, c] + [0, 2, 9, 0, c - 3] + [0, c] * (sb.rows - 2)
    assert got == want


def test_deflate_round_trip_and_sizes():
    table = geo.subband_table(64, 96, 2, [4, 32])
    idx = _sparse_plane(table, 0.1, 3)
    sym, off = rle.encode_plane(idx, table, False)
    per, whole = rle.deflate_sizes(sym, off)
    assert len(per) == len(table) and all(p > 0 for p in per)
    blob = zlib.compress(np.asarray(sym, '<i2').tobytes(), 6)
    assert len(blob) == whole
    back = np.frombuffer(zlib.decompress(blob), dtype='<i2')
    np.testing.assert_array_equal(back, sym)


def test_decoder_rejects_overlong_run():
    with pytest.raises(ValueError):
        rle.unrle_row([0, 5], 0, 3)
