"""Full-search block-matching motion estimation on the luminance channel.
Test infrastructure only.

Paper section 3.2: the luminance of the current frame is cut into 16 x 16
blocks; each block is compared with every block of the previous frame
displaced by at most W pixels in each direction ((2W + 1)^2 candidates,
the undisplaced one included), with the mean squared error as the measure;
the best candidate gives the block's motion vector.

Readings:
  * blocks tile the frame from its top-left corner: ceil(H / 16) by
    ceil(W / 16) blocks, those on the bottom and right edges cropped to the
    frame;
  * a candidate counts only if the displaced block lies wholly inside the
    previous frame, so the undisplaced block always counts;
  * luminance is taken on its 8-bit scale in steps of 1/4 (the YCoCg front
    end produces exactly such values): each value is rounded to the nearest
    quarter (halves to even) and clamped to [0, 255], and the squared errors
    are summed exactly as integers (of 4 Y). Candidates of one block have the
    same pixel count, so the smallest sum is the smallest MSE;
  * ties go to the smallest |dy| + |dx|, then the smallest dy, then the
    smallest dx;
  * a motion vector (dy, dx) says that the block at (y, x) of the current
    frame matches the block at (y + dy, x + dx) of the previous one.
"""
import numpy as np

BLOCK = 16


def quarters(a):
    """Luminance as integers 4 Y in [0, 1020]."""
    q = np.rint(np.asarray(a, dtype=np.float64) * 4.0)
    return np.clip(q, 0, 1020).astype(np.int64)


def block_grid(height, width):
    return -(-height // BLOCK), -(-width // BLOCK)


def match_block(c, p, by, bx, w):
    """Best (dy, dx, ssd) of block (by, bx); c and p are quarters() planes."""
    H, W = c.shape
    y0, x0 = by * BLOCK, bx * BLOCK
    bh, bw = min(BLOCK, H - y0), min(BLOCK, W - x0)
    blk = c[y0:y0 + bh, x0:x0 + bw]
    best = None
    for dy in range(-w, w + 1):
        for dx in range(-w, w + 1):
            if y0 + dy < 0 or x0 + dx < 0 or y0 + dy + bh > H or x0 + dx + bw > W:
                continue
            cand = p[y0 + dy:y0 + dy + bh, x0 + dx:x0 + dx + bw]
            ssd = int(((blk - cand) ** 2).sum())
            key = (ssd, abs(dy) + abs(dx), dy, dx)
            if best is None or key < best:
                best = key
    return best[2], best[3], best[0]


def block_match(cur, prev, w):
    """Motion vectors [nby][nbx][2] (dy, dx) and sums [nby][nbx] of squared
    differences of 4 Y for one frame pair."""
    c, p = quarters(cur), quarters(prev)
    nby, nbx = block_grid(*c.shape)
    mv = np.zeros((nby, nbx, 2), dtype=np.int64)
    ssd = np.zeros((nby, nbx), dtype=np.int64)
    for by in range(nby):
        for bx in range(nbx):
            dy, dx, s = match_block(c, p, by, bx, w)
            mv[by, bx] = (dy, dx)
            ssd[by, bx] = s
    return mv, ssd
