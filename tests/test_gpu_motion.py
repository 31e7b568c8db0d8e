"""GPU parity of the block-matching motion search against the oracle.

Integer work: the motion vectors and the sums of squared differences (of
4 Y) must equal the oracle's bit for bit, ties included (the oracle's order
of (sum, |dy| + |dx|, dy, dx) makes the answer unique).
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import motion
from paper_1510_00561_amd import ct, synth
from tests import clips

pytestmark = pytest.mark.gpu


def _pair(name, B, H, W):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    prev = rng.integers(0, 1021, (B, H, W)) / 4.0
    # the current frame: the previous one moved by a per-plane shift, plus
    # noise on a tenth of the pixels
    cur = np.empty_like(prev)
    for b in range(B):
        sy, sx = rng.integers(-5, 6, 2)
        cur[b] = np.roll(prev[b], (int(sy), int(sx)), axis=(0, 1))
    cur += (rng.random(cur.shape) < 0.1) * rng.integers(-8, 9, cur.shape) / 4.0
    return cur.astype(np.float32), prev.astype(np.float32)


# (name, batch, height, width, w): multiples of 16, cropped edge blocks on
# either side, a frame narrower than one block, w from 1 to 16
CASES = [
    ("w8", 2, 64, 96, 8),
    ("ragged", 2, 45, 70, 8),
    ("w1", 1, 48, 48, 1),
    ("w16", 1, 50, 66, 16),
    ("tiny", 3, 5, 9, 3),
    ("w4", 2, 33, 130, 4),
]


@pytest.mark.parametrize("name,B,H,W,w", CASES, ids=[c[0] for c in CASES])
def test_motion_search_exact(name, B, H, W, w):
    cur, prev = _pair(name, B, H, W)
    print(f"[motion] {name} B={B} H={H} W={W} w={w}", flush=True)
    mv, ssd = ct.motion_search(torch.from_numpy(cur).cuda(), torch.from_numpy(prev).cuda(), w)
    mv, ssd = mv.cpu().numpy(), ssd.cpu().numpy()
    for b in range(B):
        omv, ossd = motion.block_match(cur[b], prev[b], w)
        assert np.array_equal(mv[b], omv), b
        assert np.array_equal(ssd[b], ossd), b


def test_motion_ties_and_rounding():
    # flat frames: every candidate ties, the zero vector wins; values off the
    # quarter grid and outside [0, 255] round and clamp as in the oracle
    B, H, W, w = 2, 32, 48, 8
    rng = np.random.default_rng(3)
    prev = np.full((B, H, W), 77.0, dtype=np.float32)
    cur = prev.copy()
    cur[1] = rng.uniform(-20, 300, (H, W)).astype(np.float32)
    prev[1] = rng.uniform(-20, 300, (H, W)).astype(np.float32)
    mv, ssd = ct.motion_search(torch.from_numpy(cur).cuda(), torch.from_numpy(prev).cuda(), w)
    mv, ssd = mv.cpu().numpy(), ssd.cpu().numpy()
    assert not mv[0].any() and not ssd[0].any()
    omv, ossd = motion.block_match(cur[1], prev[1], w)
    assert np.array_equal(mv[1], omv) and np.array_equal(ssd[1], ossd)


def test_motion_full_size_sampled():
    # 15 pairs of consecutive synthetic 1080p frames (Y planes of the clip, as
    # the library's colour front end produces them), w = 8 (section 4.1): 40
    # sampled blocks per pair against the oracle, edges and corners included
    F, H, W, w = 16, 1080, 1920, 8
    ys = clips.clip_planes(F, H, W, 3)[0::3]
    print("[motion] full size 15 x 1080p pairs w=8", flush=True)
    y = torch.from_numpy(ys).cuda()
    mv, ssd = ct.motion_search(y[1:].contiguous(), y[:-1].contiguous(), w)
    mv, ssd = mv.cpu().numpy(), ssd.cpu().numpy()
    nby, nbx = motion.block_grid(H, W)
    rng = np.random.default_rng(8)
    for b in range(F - 1):
        c, p = motion.quarters(ys[b + 1]), motion.quarters(ys[b])
        picks = [(0, 0), (nby - 1, nbx - 1), (nby - 1, 0), (0, nbx - 1)]
        picks += [tuple(v) for v in np.stack([rng.integers(0, nby, 36), rng.integers(0, nbx, 36)], 1)]
        for by, bx in picks:
            dy, dx, s = motion.match_block(c, p, by, bx, w)
            assert (mv[b, by, bx, 0], mv[b, by, bx, 1], ssd[b, by, bx]) == (dy, dx, s), (b, by, bx)
    # the clip's objects move, so not every block stays put
    assert (mv != 0).any()


def test_motion_errors_and_empty():
    z = torch.zeros((0, 16, 16), dtype=torch.float32, device="cuda")
    mv, _ = ct.motion_search(z, z, 8)
    assert mv.shape == (0, 1, 1, 2)
    x = torch.zeros((1, 16, 16), dtype=torch.float32, device="cuda")
    for bad in (0, 17):
        with pytest.raises(ct.CTError):
            ct.motion_search(x, x, bad)
    mv, ssd = ct.motion_search(x, x, 2, want_ssd=False)
    assert ssd is None and not mv.cpu().numpy().any()
