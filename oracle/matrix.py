"""Explicit dense matrices of the contourlet transform, built stage by stage.

This module re-derives every stage as a matrix from the definitions, without
calling the array code of lp.py, dfb.py or ct.py, so that the product of the
stage matrices can be compared entry by entry with the array path applied to
unit vectors. It is only usable for small frames (16x16, 32x32).

Stages (section 2.1: LP, then a DFB on every bandpass, iterated on the
lowpass; readings as in geometry.py, lp.py and dfb.py):
  * reflect padding to the R x C torus;
  * LP analysis  c = D (Hbar) x,  d = x - Gbar U c, with circulant filter
    matrices, D the keep-even decimation and U its transpose;
  * DFB node on a coset with basis (v1, v2): K = (P_v2 + P_-v2 - P_v1 - P_-v1)/4
    restricted to the coset, y0 = E p(K) x, y1 = O q(-K) x;
  * the tree (tree level 1: basis (1,0),(0,1); level 2: (1,1),(-1,1) for the
    vertical cone and (1,1),(1,-1) for the horizontal cone; level t >= 3:
    (2a, -2^(t-2)), (2a+2, -2^(t-2)) vertical, coordinates swapped for
    horizontal; even child a' = 2a+1, odd child a' = 2a);
  * packing: lowpass, then levels coarse to fine, subbands by (horizontal,
    ascending a) then (vertical, descending a); horizontal subbands row
    major, vertical subbands column major.
Flattening is row major: pixel (n1, n2) of an R x C image has index n1*C + n2.
"""
import numpy as np

from . import filters


def circulant(taps, n):
    """Matrix of y[i] = sum_k taps[k] x[i - k] on a length-n torus (centred taps)."""
    centre = len(taps) // 2
    M = np.zeros((n, n))
    for idx, t in enumerate(taps):
        k = idx - centre
        for i in range(n):
            M[i, (i - k) % n] += t
    return M


def decimation(n):
    """(n/2) x n matrix keeping even samples."""
    Dm = np.zeros((n // 2, n))
    Dm[np.arange(n // 2), 2 * np.arange(n // 2)] = 1.0
    return Dm


def pad_matrix(H, W, R, C):
    """Reflect-padding matrix (R*C) x (H*W)."""
    def src(i, n):
        return i if i < n else 2 * n - 1 - i
    P = np.zeros((R * C, H * W))
    for r in range(R):
        for c in range(C):
            P[r * C + c, src(r, H) * W + src(c, W)] = 1.0
    return P


def lp_matrices(R, C, lo, up):
    """(A_c, A_d): LP analysis maps x -> c and x -> d on an R x C torus."""
    Hc = np.kron(decimation(R) @ circulant(lo, R), decimation(C) @ circulant(lo, C))
    Ug = np.kron(circulant(up, R) @ decimation(R).T, circulant(up, C) @ decimation(C).T)
    return Hc, np.eye(R * C) - Ug @ Hc


def lp_synthesis_matrices(R, C, lo, up, recon='dual'):
    """(S_c, S_d): LP synthesis x = S_c c + S_d d.

    Dual frame: x = U c + (I - U H) d, U the upsampling filter and H the
    decimating lowpass. Burt-Adelson: x = U c + d.
    """
    Hd = np.kron(decimation(R) @ circulant(lo, R), decimation(C) @ circulant(lo, C))
    Ug = np.kron(circulant(up, R) @ decimation(R).T, circulant(up, C) @ decimation(C).T)
    if recon == 'ba':
        return Ug, np.eye(R * C)
    return Ug, np.eye(R * C) - Ug @ Hd


def shift_perm(R, C, v):
    """Matrix of (S_v x)[n] = x[n + v] on the R x C torus."""
    P = np.zeros((R * C, R * C))
    for n1 in range(R):
        for n2 in range(C):
            P[n1 * C + n2, ((n1 + v[0]) % R) * C + (n2 + v[1]) % C] = 1.0
    return P


def _poly_matrix(coeffs, K):
    out = np.zeros_like(K)
    power = np.eye(K.shape[0])
    for c in coeffs:
        out += c * power
        power = power @ K
    return out


def _children(points, o, v1, v2, R, C):
    """Split coset points into (even, odd) by the parity of m1 + m2.

    Enumerates o + m1 v1 + m2 v2 over a range of (m1, m2) wide enough to
    reach every point of the torus, and checks that each point receives a
    single parity.
    """
    lim = 2 * max(R, C)
    parity = {}
    for m1 in range(-lim, lim + 1):
        for m2 in range(-lim, lim + 1):
            p = ((o[0] + m1 * v1[0] + m2 * v2[0]) % R, (o[1] + m1 * v1[1] + m2 * v2[1]) % C)
            par = (m1 + m2) % 2
            assert parity.setdefault(p, par) == par, "parity is not defined on the torus"
    assert all(p in parity for p in points), "point not on the coset"
    even = [p for p in points if parity[p] == 0]
    odd = [p for p in points if parity[p] == 1]
    return even, odd


def _canon(o, D):
    """Coset representative reduced into [0, D1) x [0, D2).

    The even sub-coset of a node is the one containing its representative,
    so the representative must be canonical: it is the smallest point of the
    coset in each coordinate.
    """
    return (o[0] % D[0], o[1] % D[1])


def _basis(cone, a, t):
    if t == 1:
        return (1, 0), (0, 1)
    if t == 2:
        return ((1, 1), (-1, 1)) if cone == 'V' else ((1, 1), (1, -1))
    m = t - 2
    if cone == 'V':
        return (2 * a, -(1 << m)), (2 * a + 2, -(1 << m))
    return (-(1 << m), 2 * a), (-(1 << m), 2 * a + 2)


def dfb_matrix(R, C, l, f0, f1):
    """DFB analysis matrix (R*C) x (R*C) with rows in packed subband order.

    Channels are tracked as point lists on the level torus together with the
    matrix mapping the level image to the channel's values at those points.
    """
    shifts = {}

    def perm(v):
        if v not in shifts:
            shifts[v] = shift_perm(R, C, v)
        return shifts[v]

    def node_split(points, M, o, v1, v2):
        idx = [p[0] * C + p[1] for p in points]
        Kfull = (perm(v2) + perm((-v2[0], -v2[1])) - perm(v1) - perm((-v1[0], -v1[1]))) / 4.0
        K = Kfull[np.ix_(idx, idx)]
        even, odd = _children(points, o, v1, v2, R, C)
        pos = {p: i for i, p in enumerate(points)}
        ie = [pos[p] for p in even]
        io = [pos[p] for p in odd]
        Me = (_poly_matrix(f0, K) @ M)[ie]
        Mo = (_poly_matrix(f1, K) @ M)[io]
        return (even, Me), (odd, Mo)

    allpts = [(i, k) for i in range(R) for k in range(C)]
    # channel record: (cone, a, points, matrix, offset)
    (pe, Me), (po, Mo) = node_split(allpts, np.eye(R * C), (0, 0), *_basis('root', 0, 1))
    chans = [('V', 0, pe, Me, (0, 0)), ('H', 0, po, Mo, (1, 0))]
    if l >= 2:
        nxt = []
        for cone, a, pts, M, o in chans:
            v1, v2 = _basis(cone, a, 2)
            (ce, Ce), (co, Co) = node_split(pts, M, o, v1, v2)
            nxt.append((cone, 0, ce, Ce, o))
            nxt.append((cone, -1, co, Co, _canon((o[0] + v1[0], o[1] + v1[1]), (2, 2))))
        chans = nxt
    for t in range(3, l + 1):
        nxt = []
        for cone, a, pts, M, o in chans:
            v1, v2 = _basis(cone, a, t)
            (ce, Ce), (co, Co) = node_split(pts, M, o, v1, v2)
            D = (2, 1 << (t - 1)) if cone == 'V' else (1 << (t - 1), 2)
            nxt.append((cone, 2 * a + 1, ce, Ce, _canon(o, D)))
            nxt.append((cone, 2 * a, co, Co, _canon((o[0] + v1[0], o[1] + v1[1]), D)))
        chans = nxt
    horiz = sorted([c for c in chans if c[0] == 'H'], key=lambda c: c[1])
    vert = sorted([c for c in chans if c[0] == 'V'], key=lambda c: -c[1])
    rows = []
    for cone, a, pts, M, o in horiz + vert:
        key = (lambda p: (p[1], p[0])) if cone == 'V' else (lambda p: (p[0], p[1]))
        order = sorted(range(len(pts)), key=lambda i: key(pts[i]))
        rows.append(M[order])
    return np.vstack(rows)


def forward_matrix(H, W, R, C, levels, dirs, kind='97'):
    """Dense matrix of the forward CT on an H x W frame (filter pair `kind`)."""
    p, q = filters.polynomials(kind)
    hbar, gbar = filters.lp_filters(kind)
    q_neg = filters.negate_argument(q)
    M = pad_matrix(H, W, R, C)
    blocks = []
    for j in range(levels):
        Rj, Cj = R >> j, C >> j
        Ac, Ad = lp_matrices(Rj, Cj, hbar, gbar)
        l = int(np.log2(dirs[j]))
        blocks.append(dfb_matrix(Rj, Cj, l, p, q_neg) @ Ad @ M)
        M = Ac @ M
    return np.vstack([M] + blocks[::-1])


def inverse_matrix(H, W, R, C, levels, dirs, kind='97', recon='dual'):
    """Dense matrix of the inverse CT (coefficients -> H x W frame)."""
    p, q = filters.polynomials(kind)
    hbar, gbar = filters.lp_filters(kind)
    p_neg = filters.negate_argument(p)
    # DFB synthesis is the exact inverse of analysis; build it as the
    # synthesis polynomial pair applied through the transpose structure:
    # Syn[g0, g1] = (Ana[g0, g1])^T because K is symmetric and E, O are
    # coordinate selections.
    sizes = [(R >> j, C >> j) for j in range(levels)]
    low_n = (R >> levels) * (C >> levels)
    band_n = [r * c for r, c in sizes]
    # coefficient blocks in packed order: lowpass, level J, ..., level 1
    offs = {}
    o = low_n
    for j in range(levels - 1, -1, -1):
        offs[j] = o
        o += band_n[j]
    ncoef = o
    # reconstruct from the coarsest level down
    Xc = np.zeros((low_n, ncoef))
    Xc[:, :low_n] = np.eye(low_n)
    for j in range(levels - 1, -1, -1):
        Rj, Cj = sizes[j]
        l = int(np.log2(dirs[j]))
        Ssyn = dfb_matrix(Rj, Cj, l, q, p_neg).T
        Dd = np.zeros((Rj * Cj, ncoef))
        Dd[:, offs[j]:offs[j] + band_n[j]] = Ssyn
        Sc, Sd = lp_synthesis_matrices(Rj, Cj, hbar, gbar, recon)
        Xc = Sc @ Xc + Sd @ Dd
    crop = np.zeros((H * W, R * C))
    for r in range(H):
        for c in range(W):
            crop[r * W + c, r * C + c] = 1.0
    return crop @ Xc
