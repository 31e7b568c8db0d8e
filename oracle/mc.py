"""Motion-compensated prediction of the contourlet components of P-frames
(paper section 3.7).

TEST INFRASTRUCTURE ONLY: the plain reference of the device kernel; the
product path never imports it.

Paper, section 3.7: the components of a P-frame are the difference between
the current frame's components and their motion-compensated prediction
from the previous frame. The prediction is made on the CT components rather
than on the raw frame (a difference of raw frames would create artificial
edges), by mapping the motion vectors of section 3.2 (16 x 16 luminance
blocks) to the scale and range of each component.

Readings:
  * vectors come from motion.block_match on the luminance: (dy, dx) of block
    (by, bx) says that the block at (y, x) of the current frame matches the
    one at (y + dy, x + dx) of the previous frame;
  * a directional subband sample (i, k) of level j, with lattice offset
    (o1, o2) and steps (s1, s2) in level-j coordinates, sits at luminance
    pixel n 2^(j-1) (o1 + s1 i, o2 + s2 k); a lowpass sample (i, k) at
    n 2^J (i, k); n is the chroma subsampling factor of the channel (1 for
    luminance);
  * the sample takes the vector of the block holding that pixel; pixels of
    the padding below or right of the frame take the last block row or
    column;
  * the vector maps to the component's grid by division by the sample
    spacing (n 2^(j-1) s1 rows, n 2^(j-1) s2 columns; n 2^J for the lowpass),
    rounded to the nearest integer with halves away from zero;
  * prediction[i][k] = previous component[(i + di) mod rows][(k + dk) mod
    cols] in natural orientation: the components are periodic, as the
    transform is;
  * the P-frame component is current - prediction on the quantised int16
    indices, modulo 2^16 (as the K-frame lowpass filter), so that the decoder
    restores current = component + prediction exactly.
"""
import numpy as np

BLOCK = 16


def round_div(a, b):
    """a / b rounded to the nearest integer, halves away from zero (b > 0)."""
    a = np.asarray(a, dtype=np.int64)
    q = (2 * np.abs(a) + b) // (2 * b)
    return np.sign(a) * q


def spacing(sb, levels, n=1):
    """Sample spacing of a component in luminance pixels: (rows, columns)."""
    if sb.k < 0:
        return n << levels, n << levels
    f = n << (sb.level - 1)
    return f * sb.s1, f * sb.s2


def sample_pixels(sb, levels, n=1):
    """Luminance pixel (y, x) of every natural sample (i, k): two rows x cols arrays."""
    i, k = np.meshgrid(np.arange(sb.rows), np.arange(sb.cols), indexing='ij')
    if sb.k < 0:
        f = n << levels
        return f * i, f * k
    f = n << (sb.level - 1)
    return f * (sb.o1 + sb.s1 * i), f * (sb.o2 + sb.s2 * k)


def component_vectors(sb, levels, mv, n=1):
    """Mapped displacement (di, dk) of every natural sample of component sb."""
    mv = np.asarray(mv)
    nby, nbx = mv.shape[:2]
    py, px = sample_pixels(sb, levels, n)
    by = np.minimum(py // BLOCK, nby - 1)
    bx = np.minimum(px // BLOCK, nbx - 1)
    sy, sx = spacing(sb, levels, n)
    return round_div(mv[by, bx, 0], sy), round_div(mv[by, bx, 1], sx)


def natural(comp, sb):
    a = np.asarray(comp)
    return a.reshape(sb.cols, sb.rows).T if sb.transposed else a.reshape(sb.rows, sb.cols)


def stored(nat, sb):
    return (nat.T if sb.transposed else nat).reshape(-1)


def predict_plane(prev, table, levels, mv, n=1):
    """Motion-compensated prediction of every component of a plane (any dtype)."""
    prev = np.asarray(prev)
    out = np.empty_like(prev)
    for sb in table:
        p = natural(prev[sb.offset:sb.offset + sb.size], sb)
        di, dk = component_vectors(sb, levels, mv, n)
        i, k = np.meshgrid(np.arange(sb.rows), np.arange(sb.cols), indexing='ij')
        out[sb.offset:sb.offset + sb.size] = stored(p[(i + di) % sb.rows, (k + dk) % sb.cols], sb)
    return out


def residual_plane(cur, prev, table, levels, mv, n=1):
    """P-frame components: current - prediction, int16 modulo 2^16."""
    pred = predict_plane(np.asarray(prev, dtype=np.int64), table, levels, mv, n)
    return (np.asarray(cur, dtype=np.int64) - pred).astype(np.int16)


def restore_plane(resid, prev, table, levels, mv, n=1):
    """Decoder side: component + prediction, int16 modulo 2^16."""
    pred = predict_plane(np.asarray(prev, dtype=np.int64), table, levels, mv, n)
    return (np.asarray(resid, dtype=np.int64) + pred).astype(np.int16)
