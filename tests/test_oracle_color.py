"""Pins of the colour, chroma and K-frame lowpass stages (sections 2.3, 3.1, 3.7)."""
import numpy as np
import pytest

from oracle import color


def _rgb(h, w, seed):
    return np.random.default_rng(seed).integers(0, 256, size=(h, w, 3)).astype(np.uint8)


def test_table1_known_colours():
    # equations (1)-(3) at the primaries, white and black, computed by hand
    cases = {
        (255, 0, 0): (63.75, 127.5, -63.75),
        (0, 255, 0): (127.5, 0.0, 127.5),
        (0, 0, 255): (63.75, -127.5, -63.75),
        (255, 255, 255): (255.0, 0.0, 0.0),
        (0, 0, 0): (0.0, 0.0, 0.0),
        (100, 50, 20): (55.0, 40.0, -5.0),
    }
    for rgb, want in cases.items():
        y, co, cg = color.rgb_to_ycocg(np.array(rgb, dtype=np.float64).reshape(1, 1, 3))
        assert (float(y[0, 0]), float(co[0, 0]), float(cg[0, 0])) == want


def test_table1_round_trip_exact():
    # Y, Co, Cg of 8-bit RGB are quarter integers, so (4)-(6) invert (1)-(3) exactly
    rgb = _rgb(17, 23, 1)
    y, co, cg = color.rgb_to_ycocg(rgb)
    for a in (y, co, cg):
        assert np.array_equal(a * 4, np.round(a * 4))
    back = color.ycocg_to_rgb(y, co, cg)
    assert np.array_equal(back, rgb.astype(np.float64))


def test_chroma_range_section31():
    # equations (2)-(3): Co and Cg of 8-bit RGB lie within [-127.5, 127.5] (section 3.1
    # rounds this to [-127, 127]), so +127 maps them to [-0.5, 254.5]; the extremes occur
    rgb = np.array([[[255, 0, 0], [0, 0, 255], [0, 255, 0], [255, 0, 255]]], dtype=np.float64)
    _, co, cg = color.rgb_to_ycocg(rgb)
    assert co.max() == 127.5 and co.min() == -127.5
    assert cg.max() == 127.5 and cg.min() == -127.5


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_subsample_keeps_the_grid(n):
    c = np.arange(7 * 10, dtype=np.float64).reshape(7, 10)
    s = color.subsample(c, n)
    assert s.shape == (-(-7 // n), -(-10 // n))
    for i in range(s.shape[0]):
        for j in range(s.shape[1]):
            assert s[i, j] == c[n * i, n * j] + 127


@pytest.mark.parametrize("n", [1, 2, 4])
def test_upsample_exact_on_samples_and_planes(n):
    h, w = 9, 13
    rng = np.random.default_rng(n)
    cs = rng.uniform(0, 255, size=(-(-h // n), -(-w // n)))
    up = color.upsample(cs, n, h, w)
    # the kept samples come back unchanged (minus the offset)
    assert np.allclose(up[::n, ::n], cs - 127, atol=1e-12)
    # bilinear interpolation reproduces an affine function between samples
    ii, jj = np.meshgrid(np.arange(cs.shape[0]), np.arange(cs.shape[1]), indexing="ij")
    affine = 3.0 + 2.0 * (n * ii) - 0.5 * (n * jj)
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    want = 3.0 + 2.0 * yy - 0.5 * xx - 127
    got = color.upsample(affine, n, h, w)
    inside = (yy <= n * (cs.shape[0] - 1)) & (xx <= n * (cs.shape[1] - 1))
    assert np.allclose(got[inside], want[inside], atol=1e-12)
    # past the last sample the last one is held
    last_row = n * (cs.shape[0] - 1)
    assert np.allclose(got[last_row:, 0], got[last_row, 0])


def test_frame_round_trip_full_chroma():
    rgb = _rgb(12, 20, 3)
    y, cos, cgs = color.encode_frame(rgb, 1)
    assert np.array_equal(color.decode_frame(y, cos, cgs, 1), rgb.astype(np.float64))


def test_frame_round_trip_smooth_chroma():
    # chroma that is affine in the pixel position survives subsampling by 2 when the
    # last row and column are kept samples (9 = 2*4 + 1, 11 = 2*5 + 1)
    h, w = 9, 11
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    rgb = np.stack([100 + 4 * yy, 120 + 2 * xx, 90 + yy + xx], axis=-1).astype(np.float64)
    y, cos, cgs = color.encode_frame(rgb, 2)
    back = color.decode_frame(y, cos, cgs, 2)
    assert np.allclose(back, rgb, atol=1e-9)


def test_lowpass_column_diff_worked():
    q = np.array([[10, 12, 0],
                  [11, 12, -3],
                  [13, 10, -3]])
    d = color.lowpass_column_diff(q)
    assert d.tolist() == [[10, 12, 0], [1, 0, -3], [2, -2, 0]]
    assert np.array_equal(color.lowpass_column_undiff(d), q)


def test_lowpass_column_diff_constant_columns():
    # neighbouring equal values give zeros below the first row (section 3.7)
    q = np.tile(np.array([[5, 9, 200]]), (6, 1))
    d = color.lowpass_column_diff(q)
    assert np.array_equal(d[0], q[0]) and not d[1:].any()


def test_lowpass_column_round_trip_random():
    q = np.random.default_rng(5).integers(0, 256, size=(17, 30))
    assert np.array_equal(color.lowpass_column_undiff(color.lowpass_column_diff(q)), q)
