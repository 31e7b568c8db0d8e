"""Directional filter bank (DFB): a tree of two-channel quincunx fan filter banks.

Paper: section 2.1. The DFB splits each LP bandpass image into 2^l subbands
with wedge-shaped frequency support, and uses the 9-7 filters. The
construction of the fan filters and the tree geometry are a reading; see
geometry.py for the tree.

Fan filter bank (one tree node), operator form. The channel lives on a
lattice coset with basis (v1, v2). Let S_v be the shift (S_v x)[n] = x[n + v]
on the torus, and let

    K = (S_v2 + S_-v2 - S_v1 - S_-v1) / 4,

a self-adjoint operator whose symbol is (cos(w.v2) - cos(w.v1)) / 2. E and O
are the projections onto the even and odd sub-cosets {o + m1 v1 + m2 v2 :
m1 + m2 even / odd}. With p, q the 9-7 pair as polynomials in cos(w)
(filters.py):

    analysis    y0 = E p(K) x,   y1 = O q(-K) x
    synthesis   x  = q(K) E y0 + p(-K) O y1

This is the 9-7 pair carried from 1-D to the fan geometry by the change of
variable cos(w) -> K (transformation of variables). Perfect reconstruction
follows from p(t) q(t) + p(-t) q(-t) = 2 and Mod K Mod = -K, where Mod is the
+-1 parity modulation.

The functions are generic in the polynomial pair: the forward DFB is
analysis with (p, q(-t)), the inverse is synthesis with (q, p(-t)); the
transposes swap the roles (see ct.py).

Representation: tree levels 1 and 2 act on full-size level images, with
zeros off the channel's coset. From tree level 3 on, every channel lives on
o + diag(D) Z^2 and is held as its compact array X[i, k] = x[o + D (i, k)].
Subbands are returned in their natural orientation.
"""
import numpy as np

from . import geometry as geo


def apply_poly(coeffs, op, x):
    """sum_k coeffs[k] op^k (x), evaluated by Horner's rule."""
    y = coeffs[-1] * x
    for c in coeffs[-2::-1]:
        y = op(y) + c * x
    return y


def _roll(x, v):
    """(S_v x)[n] = x[n + v] on the torus of x's shape."""
    return np.roll(x, (-v[0], -v[1]), axis=(0, 1))


def fan_kernel(v1, v2):
    """K as a function on arrays, for shifts v1, v2 in array coordinates."""
    m1 = (-v1[0], -v1[1])
    m2 = (-v2[0], -v2[1])

    def op(x):
        return (_roll(x, v2) + _roll(x, m2) - _roll(x, v1) - _roll(x, m1)) / 4.0
    return op


def _coset_parity_full(shape, o, v1, v2):
    """(member, parity) masks for the coset o + span(v1, v2) on a full torus.

    parity is m1 + m2 mod 2 where n - o = m1 v1 + m2 v2. Solved with the
    integer adjugate; points with a non-integer solution are not members.
    """
    R, C = shape
    n1, n2 = np.meshgrid(np.arange(R), np.arange(C), indexing='ij')
    d1, d2 = n1 - o[0], n2 - o[1]
    det = v1[0] * v2[1] - v2[0] * v1[1]
    # adj(B) (n - o), B = [v1 v2] as columns
    a1 = v2[1] * d1 - v2[0] * d2
    a2 = -v1[1] * d1 + v1[0] * d2
    member = (a1 % abs(det) == 0) & (a2 % abs(det) == 0)
    parity = ((a1 // det + a2 // det) % 2).astype(bool)
    # the parity must be a function on the torus: shifting by a period
    # (R, 0) or (0, C) must keep m1 + m2 even
    for per in ((R, 0), (0, C)):
        p1 = v2[1] * per[0] - v2[0] * per[1]
        p2 = -v1[1] * per[0] + v1[0] * per[1]
        assert p1 % det == 0 and p2 % det == 0 and (p1 // det + p2 // det) % 2 == 0, \
            "torus period is not in the even sub-lattice"
    return member, parity


def _compact_parity(shape, u1, u2):
    """Parity m1 + m2 of compact index (i, k) = m1 u1 + m2 u2 (det = +-1)."""
    det = u1[0] * u2[1] - u2[0] * u1[1]
    assert abs(det) == 1
    n, kk = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing='ij')
    m1 = (u2[1] * n - u2[0] * kk) * det
    m2 = (-u1[1] * n + u1[0] * kk) * det
    for per in ((shape[0], 0), (0, shape[1])):
        q1 = (u2[1] * per[0] - u2[0] * per[1]) * det
        q2 = (-u1[1] * per[0] + u1[0] * per[1]) * det
        assert (q1 + q2) % 2 == 0, "compact period breaks the parity"
    return ((m1 + m2) % 2).astype(bool)


def _qfb_full(x, o, v1, v2, f0, f1):
    """Analysis node on a full-size image; returns (y0, y1), zero off-coset."""
    member, odd = _coset_parity_full(x.shape, o, v1, v2)
    K = fan_kernel(v1, v2)
    y0 = np.where(member & ~odd, apply_poly(f0, K, x), 0.0)
    y1 = np.where(member & odd, apply_poly(f1, K, x), 0.0)
    return y0, y1


def _qfb_full_syn(y0, y1, o, v1, v2, g0, g1):
    member, odd = _coset_parity_full(y0.shape, o, v1, v2)
    K = fan_kernel(v1, v2)
    e = np.where(member & ~odd, y0, 0.0)
    od = np.where(member & odd, y1, 0.0)
    return apply_poly(g0, K, e) + apply_poly(g1, K, od)


def _compact_shift(v, D):
    assert v[0] % D[0] == 0 and v[1] % D[1] == 0
    return (v[0] // D[0], v[1] // D[1])


def _child_index(parent, child, shape_child):
    """Parent compact indices of every element of a child array."""
    i, k = np.meshgrid(np.arange(shape_child[0]), np.arange(shape_child[1]),
                       indexing='ij')
    n1 = child.o[0] + child.D[0] * i - parent.o[0]
    n2 = child.o[1] + child.D[1] * k - parent.o[1]
    assert np.all(n1 % parent.D[0] == 0) and np.all(n2 % parent.D[1] == 0)
    return n1 // parent.D[0], n2 // parent.D[1]


def _extract_coset(img, node):
    """Compact array of a full-size image on node's coset o + diag(D) Z^2."""
    return img[node.o[0]::node.D[0], node.o[1]::node.D[1]].copy()


def _embed_coset(arr, node, shape):
    img = np.zeros(shape, dtype=np.float64)
    img[node.o[0]::node.D[0], node.o[1]::node.D[1]] = arr
    return img


def dfb_analysis(d, l, f0, f1):
    """DFB analysis of a level image `d` into 2^l subbands (natural orientation).

    f0, f1: polynomial coefficient arrays of the even and odd channel filters
    of every node (forward DFB: f0 = p, f1 = q(-t)).
    Returns the list of subband arrays in subband order.
    """
    d = np.asarray(d, dtype=np.float64)
    tree = geo.tree_levels(l)
    shape = d.shape
    # tree level 1 on the full image
    v1, v2 = geo.split_basis(tree[0][0], 1)
    vert, horz = _qfb_full(d, (0, 0), v1, v2, f0, f1)
    # tree level 2: vertical on the quincunx lattice, horizontal on its coset
    hnode, vnode = tree[1]
    v_even, v_odd = _qfb_full(vert, vnode.o, *geo.split_basis(vnode, 2), f0, f1)
    h_even, h_odd = _qfb_full(horz, hnode.o, *geo.split_basis(hnode, 2), f0, f1)
    level2_img = {('H', -1): h_odd, ('H', 0): h_even, ('V', 0): v_even, ('V', -1): v_odd}
    chans = {}
    for node in tree[2]:
        chans[(node.cone, node.a)] = _extract_coset(level2_img[(node.cone, node.a)], node)
    for t in range(3, l + 1):
        nxt = {}
        for parent, even, odd in _pairs(tree, t):
            X = chans[(parent.cone, parent.a)]
            v1, v2 = geo.split_basis(parent, t)
            u1, u2 = _compact_shift(v1, parent.D), _compact_shift(v2, parent.D)
            K = fan_kernel(u1, u2)
            par = _compact_parity(X.shape, u1, u2)
            Y0 = apply_poly(f0, K, X)
            Y1 = apply_poly(f1, K, X)
            for child, Y, want in ((even, Y0, False), (odd, Y1, True)):
                cshape = (shape[0] // child.D[0], shape[1] // child.D[1])
                pi, pk = _child_index(parent, child, cshape)
                assert np.all(par[pi, pk] == want)
                nxt[(child.cone, child.a)] = Y[pi, pk]
        chans = nxt
    return [chans[(n.cone, n.a)] for n in tree[l]]


def _pairs(tree, t):
    """(parent, even child, odd child) triples for the split at tree level t."""
    out = []
    children = {(n.cone, n.a): n for n in tree[t]}
    for parent in tree[t - 1]:
        even = children[(parent.cone, 2 * parent.a + 1)]
        odd = children[(parent.cone, 2 * parent.a)]
        out.append((parent, even, odd))
    return out


def dfb_synthesis(subbands, l, shape, g0, g1):
    """Inverse tree: rebuild the level image from 2^l subbands.

    g0, g1: polynomials applied to the even and odd channels of every node
    (inverse DFB: g0 = q, g1 = p(-t)).
    """
    tree = geo.tree_levels(l)
    chans = {(n.cone, n.a): np.asarray(s, dtype=np.float64)
             for n, s in zip(tree[l], subbands)}
    for t in range(l, 2, -1):
        nxt = {}
        for parent, even, odd in _pairs(tree, t):
            pshape = (shape[0] // parent.D[0], shape[1] // parent.D[1])
            v1, v2 = geo.split_basis(parent, t)
            u1, u2 = _compact_shift(v1, parent.D), _compact_shift(v2, parent.D)
            K = fan_kernel(u1, u2)
            E = np.zeros(pshape)
            O = np.zeros(pshape)
            for child, dst in ((even, E), (odd, O)):
                cshape = (shape[0] // child.D[0], shape[1] // child.D[1])
                pi, pk = _child_index(parent, child, cshape)
                dst[pi, pk] = chans[(child.cone, child.a)]
            nxt[(parent.cone, parent.a)] = apply_poly(g0, K, E) + apply_poly(g1, K, O)
        chans = nxt
    # tree level 2 -> 1 on full images
    nodes2 = {(n.cone, n.a): n for n in tree[2]}
    img = {key: _embed_coset(chans[key], nodes2[key], shape) for key in chans}
    hnode, vnode = tree[1]
    vert = _qfb_full_syn(img[('V', 0)], img[('V', -1)], vnode.o,
                         *geo.split_basis(vnode, 2), g0, g1)
    horz = _qfb_full_syn(img[('H', 0)], img[('H', -1)], hnode.o,
                         *geo.split_basis(hnode, 2), g0, g1)
    v1, v2 = geo.split_basis(tree[0][0], 1)
    return _qfb_full_syn(vert, horz, (0, 0), v1, v2, g0, g1)
