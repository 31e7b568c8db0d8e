"""Encoder front and back stages around the transform: colour space, chroma
subsampling, and the K-frame lowpass filtering. Test infrastructure only.

Paper:
  * section 2.3, Table I, equations (1)-(6): RGB to YCoCg and back;
  * section 3.1: the chrominance channels are subsampled by a user-defined
    factor N and shifted by +127 into [0, 255]; the decoder subtracts 127 and
    fills the missing chrominance values by bilinear interpolation from the
    four neighbouring samples;
  * section 3.7 (K-frames): down every column of the quantised lowpass
    component, each element is replaced by its difference with the element
    above it (lossless).

Readings (FP64 throughout):
  * RGB frames are 8 bits per channel, stored interleaved [H][W][3];
  * subsampling keeps the samples at (N i, N j), giving ceil(H / N) by
    ceil(W / N) chroma planes (N = 1 keeps everything);
  * bilinear upsampling places sample (i, j) at pixel (N i, N j); pixel
    (y, x) interpolates between samples floor(y / N) and the next one with
    weight (y mod N) / N, and likewise along x; past the last sample the
    last one is repeated. The +127 offset is removed after interpolating;
  * the decoder returns floating-point RGB (no rounding or clamping);
  * the first row of the lowpass is kept as is; the differences are exact
    integers (indices stay within int16);
  * section 3.1 gives [-127, 127] as the chroma range, but equations (2)
    and (3) reach -127.5 and +127.5 for 8-bit input, so the offset chroma
    lies in [-0.5, 254.5]; it is kept as a float, not clipped.
"""
import numpy as np

CHROMA_OFFSET = 127.0


def rgb_to_ycocg(rgb):
    """Table I equations (1)-(3) on an [H][W][3] array; returns Y, Co, Cg planes."""
    rgb = np.asarray(rgb, dtype=np.float64)
    r, g, b = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    y = r / 4 + g / 2 + b / 4
    co = r / 2 - b / 2
    cg = -r / 4 + g / 2 - b / 4
    return y, co, cg


def ycocg_to_rgb(y, co, cg):
    """Table I equations (4)-(6); returns an [H][W][3] array."""
    y, co, cg = (np.asarray(a, dtype=np.float64) for a in (y, co, cg))
    r = y + co - cg
    g = y + cg
    b = y - co - cg
    return np.stack([r, g, b], axis=-1)


def subsample(c, n):
    """Section 3.1: keep every n-th sample in each direction, then add 127."""
    c = np.asarray(c, dtype=np.float64)
    return c[::n, ::n] + CHROMA_OFFSET


def upsample_pixel(cs, n, yy, xx):
    """Section 3.1, decoder: the chroma value at pixel (yy, xx), bilinear
    between the four kept samples around it, with the 127 offset removed."""
    hs, ws = cs.shape
    i0 = yy // n
    fy = (yy - n * i0) / n
    i1 = min(i0 + 1, hs - 1)
    j0 = xx // n
    fx = (xx - n * j0) / n
    j1 = min(j0 + 1, ws - 1)
    v = ((1 - fy) * ((1 - fx) * float(cs[i0, j0]) + fx * float(cs[i0, j1]))
         + fy * ((1 - fx) * float(cs[i1, j0]) + fx * float(cs[i1, j1])))
    return v - CHROMA_OFFSET


def upsample(cs, n, height, width):
    """upsample_pixel over a height x width plane."""
    cs = np.asarray(cs, dtype=np.float64)
    out = np.empty((height, width))
    for yy in range(height):
        for xx in range(width):
            out[yy, xx] = upsample_pixel(cs, n, yy, xx)
    return out


def encode_frame(rgb, n):
    """RGB frame -> (Y plane, Co and Cg planes subsampled and offset)."""
    y, co, cg = rgb_to_ycocg(rgb)
    return y, subsample(co, n), subsample(cg, n)


def decode_frame(y, cos, cgs, n):
    """(Y, subsampled Co and Cg) -> RGB frame."""
    h, w = np.asarray(y).shape
    return ycocg_to_rgb(y, upsample(cos, n, h, w), upsample(cgs, n, h, w))


def lowpass_column_diff(q):
    """Section 3.7: each element minus the element above it, down every column."""
    q = np.asarray(q, dtype=np.int64)
    out = q.copy()
    out[1:, :] = q[1:, :] - q[:-1, :]
    return out


def lowpass_column_undiff(d):
    """Inverse of lowpass_column_diff: running sums down every column."""
    d = np.asarray(d, dtype=np.int64)
    return np.cumsum(d, axis=0)
