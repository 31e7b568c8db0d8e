"""Contourlet transform: LP + DFB per level, padding, packing and adjoints.

Paper: section 2.1 (contourlet filter bank = LP, then a DFB on each bandpass,
iterated on the lowpass), section 3.3 (output = coarsest lowpass plus the
directional subbands of every scale).

forward(x):  pad to the R x C torus, then for j = 1..J
               (c_j, d_j) = LP analysis of c_{j-1}      (c_0 = padded frame)
               subbands_j = DFB analysis of d_j with 2^(l_j) directions
             and pack [c_J, subbands_J, ..., subbands_1] (geometry.py).
inverse(c):  unpack, then for j = J..1
               d_j = DFB synthesis of subbands_j
               c_{j-1} = dual-frame LP synthesis of (c_j, d_j)
             and crop c_0 to H x W.

Adjoints (for the differentiable form). With A = forward and S = inverse,
written as products of stage operators, the transposes are the same stages
in reverse order with every stage transposed:
  * LP analysis (lo, up) transposes to LP synthesis with (up, lo), and dual
    LP synthesis (lo, up) transposes to LP analysis with (up, lo);
  * DFB analysis with (f0, f1) transposes to DFB synthesis with (f0, f1),
    and synthesis with (g0, g1) to analysis with (g0, g1), because K is
    self-adjoint and E, O are orthogonal projections;
  * padding by reflection transposes to folding the mirrored rows and
    columns back onto their sources; cropping transposes to zero padding.

Variants (not the paper's choice; section 2.1 names the 9-7 pair and the
LP's usual reconstruction is not specified beyond perfect reconstruction):
every function takes `filters` ('97' the paper's pair, '53' the LeGall 5/3
pair, filters.py) and the inverse and its adjoint take `recon` ('dual' the
dual-frame LP synthesis, 'ba' the Burt-Adelson one, lp.py). The forward
transform and its adjoint do not depend on `recon`.
"""
import numpy as np

from . import dfb
from . import filters
from . import geometry as geo
from . import lp


def _pad(x, R, C):
    """Reflect-pad an H x W image to R x C: x[H + i] = x[H - 1 - i]."""
    H, W = x.shape
    rows = np.array([r if r < H else 2 * H - 1 - r for r in range(R)])
    cols = np.array([c if c < W else 2 * W - 1 - c for c in range(C)])
    return x[np.ix_(rows, cols)]


def _pad_adjoint(y, H, W):
    """Transpose of _pad: each padded sample is added back onto its source."""
    R, C = y.shape
    rows = np.array([r if r < H else 2 * H - 1 - r for r in range(R)])
    cols = np.array([c if c < W else 2 * W - 1 - c for c in range(C)])
    out = np.zeros((H, W))
    np.add.at(out, (rows[:, None], cols[None, :]), y)
    return out


def _filters(kind='97'):
    p, q = filters.polynomials(kind)
    hbar, gbar = filters.lp_filters(kind)
    return p, q, hbar, gbar


RECONS = ('dual', 'ba')


def _neg(poly):
    return filters.negate_argument(poly)


def pack(lowpass, levels_subbands, table):
    """Packed coefficient vector from the lowpass and per-level subband lists.

    levels_subbands[j - 1] holds the natural-orientation subbands of level j.
    """
    out = np.zeros(table[-1].offset + table[-1].size)
    out[:table[0].size] = lowpass.ravel()
    for sb in table[1:]:
        arr = levels_subbands[sb.level - 1][sb.k]
        assert arr.shape == (sb.rows, sb.cols)
        out[sb.offset:sb.offset + sb.size] = (arr.T if sb.transposed else arr).ravel()
    return out


def unpack(vec, table, levels):
    """Inverse of pack: (lowpass, levels_subbands)."""
    vec = np.asarray(vec, dtype=np.float64)
    low = table[0]
    lowpass = vec[:low.size].reshape(low.rows, low.cols)
    subs = [[] for _ in range(levels)]
    for sb in table[1:]:
        seg = vec[sb.offset:sb.offset + sb.size]
        arr = seg.reshape(sb.cols, sb.rows).T if sb.transposed else seg.reshape(sb.rows, sb.cols)
        subs[sb.level - 1].append(arr)
    return lowpass, subs


def forward(x, levels, dirs, filters='97'):
    """Forward CT of one H x W plane; returns the packed FP64 coefficient vector."""
    x = np.asarray(x, dtype=np.float64)
    H, W = x.shape
    table = geo.subband_table(H, W, levels, dirs)
    R, C = geo.padded_size(H, W, levels, dirs)
    p, q, hbar, gbar = _filters(filters)
    c = _pad(x, R, C)
    subs = []
    for j in range(1, levels + 1):
        c, d = lp.lp_analysis(c, hbar, gbar)
        l = geo.log2_exact(dirs[j - 1])
        subs.append(dfb.dfb_analysis(d, l, p, _neg(q)))
    return pack(c, subs, table)


def inverse(vec, height, width, levels, dirs, filters='97', recon='dual'):
    """Inverse CT of one packed coefficient vector; returns the H x W plane."""
    assert recon in RECONS
    table = geo.subband_table(height, width, levels, dirs)
    R, C = geo.padded_size(height, width, levels, dirs)
    p, q, hbar, gbar = _filters(filters)
    c, subs = unpack(vec, table, levels)
    for j in range(levels, 0, -1):
        Rj, Cj = geo.level_size(R, C, j)
        l = geo.log2_exact(dirs[j - 1])
        d = dfb.dfb_synthesis(subs[j - 1], l, (Rj, Cj), q, _neg(p))
        c = lp.lp_synthesis(c, d, hbar, gbar) if recon == 'dual' else lp.lp_synthesis_ba(c, d, gbar)
    return c[:height, :width].copy()


def forward_adjoint(gvec, height, width, levels, dirs, filters='97'):
    """Transpose of forward: maps a coefficient-space vector to an H x W plane."""
    table = geo.subband_table(height, width, levels, dirs)
    R, C = geo.padded_size(height, width, levels, dirs)
    p, q, hbar, gbar = _filters(filters)
    c, subs = unpack(gvec, table, levels)
    for j in range(levels, 0, -1):
        Rj, Cj = geo.level_size(R, C, j)
        l = geo.log2_exact(dirs[j - 1])
        d = dfb.dfb_synthesis(subs[j - 1], l, (Rj, Cj), p, _neg(q))
        # transpose of LP analysis (hbar, gbar) = LP synthesis (gbar, hbar)
        c = lp.lp_synthesis(c, d, gbar, hbar)
    return _pad_adjoint(c, height, width)


def inverse_adjoint(gplane, height, width, levels, dirs, filters='97', recon='dual'):
    """Transpose of inverse: maps an H x W plane to a coefficient-space vector."""
    assert recon in RECONS
    table = geo.subband_table(height, width, levels, dirs)
    R, C = geo.padded_size(height, width, levels, dirs)
    p, q, hbar, gbar = _filters(filters)
    c = np.zeros((R, C))
    c[:height, :width] = np.asarray(gplane, dtype=np.float64)
    subs = []
    for j in range(1, levels + 1):
        if recon == 'dual':
            # transpose of dual LP synthesis (hbar, gbar) = LP analysis (gbar, hbar)
            c, d = lp.lp_analysis(c, gbar, hbar)
        else:
            c, d = lp.lp_synthesis_ba_adjoint(c, gbar)
        l = geo.log2_exact(dirs[j - 1])
        subs.append(dfb.dfb_analysis(d, l, q, _neg(p)))
    return pack(c, subs, table)
