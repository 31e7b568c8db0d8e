"""Pins of the full-search block matcher (section 3.2)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import motion


def _frame(h, w, seed):
    return np.random.default_rng(seed).integers(0, 256, size=(h, w)).astype(np.float64)


@pytest.mark.parametrize("sy,sx", [(0, 0), (3, -5), (-8, 8), (-1, 2)])
def test_known_shift_is_found(sy, sx):
    # cur(y, x) = prev(y + sy, x + sx): every block whose displaced copy lies
    # inside the frame has a zero-error candidate at (sy, sx), unique on noise
    w = 8
    prev = _frame(64, 80, 1)
    cur = np.zeros_like(prev)
    for y in range(64):
        for x in range(80):
            yy, xx = y + sy, x + sx
            cur[y, x] = prev[yy, xx] if 0 <= yy < 64 and 0 <= xx < 80 else 0.0
    mv, ssd = motion.block_match(cur, prev, w)
    for by in range(4):
        for bx in range(5):
            y0, x0 = 16 * by, 16 * bx
            if 0 <= y0 + sy and y0 + sy + 16 <= 64 and 0 <= x0 + sx and x0 + sx + 16 <= 80:
                assert tuple(mv[by, bx]) == (sy, sx) and ssd[by, bx] == 0


def test_identical_and_constant_frames():
    f = _frame(40, 50, 2)
    mv, ssd = motion.block_match(f, f, 4)
    assert not mv.any() and not ssd.any()
    c = np.full((32, 32), 77.0)
    mv, ssd = motion.block_match(c, c, 8)   # every candidate ties at zero: (0, 0) wins
    assert not mv.any() and not ssd.any()


def test_tie_order():
    # columns alternate between two values and rows are all alike: with cur one
    # column ahead of prev, every odd dx (any dy) is exact; |dy| + |dx| = 1 leaves
    # (0, -1) and (0, 1), and the smaller dx wins
    prev = np.tile(np.array([10.0, 200.0]), (48, 24))
    cur = np.tile(np.array([200.0, 10.0]), (48, 24))
    mv, ssd = motion.block_match(cur, prev, 3)
    assert (mv[1, 1] == (0, -1)).all() and ssd[1, 1] == 0
    # constant along columns too, with a one-row offset of a two-row period: now
    # dy = +-1 tie at dx = 0, and dy = -1 wins
    prev2 = np.tile(np.array([[10.0], [200.0]]), (24, 48))
    cur2 = np.tile(np.array([[200.0], [10.0]]), (24, 48))
    mv2, _ = motion.block_match(cur2, prev2, 3)
    assert tuple(mv2[1, 1]) == (-1, 0)


def test_candidates_stay_inside():
    # corner blocks can only move inward; edge blocks are cropped (40 x 50 frame)
    cur, prev = _frame(40, 50, 3), _frame(40, 50, 4)
    mv, _ = motion.block_match(cur, prev, 8)
    nby, nbx = motion.block_grid(40, 50)
    assert (nby, nbx) == (3, 4)
    for by in range(nby):
        for bx in range(nbx):
            y0, x0 = 16 * by, 16 * bx
            bh, bw = min(16, 40 - y0), min(16, 50 - x0)
            dy, dx = mv[by, bx]
            assert 0 <= y0 + dy and y0 + dy + bh <= 40 and 0 <= x0 + dx and x0 + dx + bw <= 50
            assert abs(dy) <= 8 and abs(dx) <= 8


def test_costs_agree_with_correlation():
    # SSD(d) = sum c^2 + sum p_d^2 - 2 sum c p_d, with the cross term from a 2-D
    # correlation: an independent route to every candidate's cost
    cur, prev = _frame(48, 48, 5), _frame(48, 48, 6)
    c, p = motion.quarters(cur), motion.quarters(prev)
    w = 6
    for by, bx in [(1, 1), (0, 2), (2, 0)]:
        y0, x0 = 16 * by, 16 * bx
        blk = c[y0:y0 + 16, x0:x0 + 16]
        xc = correlate2d(p, blk, mode="valid")              # xc[y, x] = sum blk * p[y:y+16, x:x+16]
        box = correlate2d(p * p, np.ones((16, 16), dtype=np.int64), mode="valid")
        best = None
        for dy in range(-w, w + 1):
            for dx in range(-w, w + 1):
                y, x = y0 + dy, x0 + dx
                if y < 0 or x < 0 or y + 16 > 48 or x + 16 > 48:
                    continue
                s = int((blk * blk).sum() + box[y, x] - 2 * xc[y, x])
                key = (s, abs(dy) + abs(dx), dy, dx)
                best = key if best is None or key < best else best
        dy, dx, s = motion.match_block(c, p, by, bx, w)
        assert (dy, dx, s) == (best[2], best[3], best[0])


def test_quarter_rounding_and_clamp():
    q = motion.quarters(np.array([0.125, 0.375, 254.9, 300.0, -3.0, 12.25]))
    assert q.tolist() == [0, 2, 1020, 1020, 0, 49]
