"""Pins of the DFB (section 2.1: 2^l wedge subbands, 9-7 filters, perfect reconstruction)."""
import json
import os

import numpy as np
import pytest

from oracle import dfb, filters
from oracle import geometry as geo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pq():
    p, q = filters.cdf97_polynomials()
    return p, q


def _fwd(d, l):
    p, q = _pq()
    return dfb.dfb_analysis(d, l, p, filters.negate_argument(q))


def _inv(subs, l, shape):
    p, q = _pq()
    return dfb.dfb_synthesis(subs, l, shape, q, filters.negate_argument(p))


@pytest.mark.parametrize("shape,l", [((8, 8), 2), ((16, 16), 3), ((32, 64), 4), ((64, 64), 5), ((128, 64), 6)])
def test_dfb_perfect_reconstruction(shape, l):
    d = np.random.default_rng(11).uniform(-128, 128, shape)
    subs = _fwd(d, l)
    assert len(subs) == 2 ** l
    assert sum(s.size for s in subs) == d.size
    np.testing.assert_allclose(_inv(subs, l, shape), d, atol=1e-10)


def _lifting_dfb(d, l, c):
    """DFB by lifting with the published 9-7 lifting constants.

    An independent algorithm for the same linear map: every node is four
    lifting steps (predict odd, update even, predict, update) with the
    neighbour sum N = 2K, then even *= zeta, odd /= zeta.
    Tree levels 1 and 2 run on the full image (parity n1 + n2, then n2);
    deeper levels on compact arrays with the sheared neighbourhoods of the
    node bases.
    """
    al, be, ga, de, ze = c["alpha"], c["beta"], c["gamma"], c["delta"], c["zeta"]

    def lift(z, odd, N):
        for coef, upd in ((al, odd), (be, ~odd), (ga, odd), (de, ~odd)):
            z = z + np.where(upd, coef * N(np.where(upd, 0.0, z)), 0.0)
        return np.where(odd, z / ze, z * ze)

    def sh(x, a, b):  # x[i + a, k + b]
        return np.roll(x, (-a, -b), axis=(0, 1))

    z = np.asarray(d, dtype=np.float64)
    R, C = z.shape
    n1, n2 = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    # tree level 1: v1 = (1,0), v2 = (0,1)
    z = lift(z, (n1 + n2) % 2 == 1, lambda x: (sh(x, 0, 1) + sh(x, 0, -1) - sh(x, 1, 0) - sh(x, -1, 0)) / 2)
    # tree level 2: both cones at once, parity n2, diagonal neighbours
    z = lift(z, n2 % 2 == 1, lambda x: (sh(x, -1, 1) + sh(x, 1, -1) - sh(x, 1, 1) - sh(x, -1, -1)) / 2)
    chans = {("H", -1): z[0::2, 1::2], ("H", 0): z[1::2, 0::2], ("V", 0): z[0::2, 0::2], ("V", -1): z[1::2, 1::2]}
    for t in range(3, l + 1):
        nxt = {}
        for (cone, a), X in chans.items():
            if cone == "H":   # rows split; neighbours (-1, a), (-1, a+1) and mirrors
                rows = np.arange(X.shape[0])[:, None] % 2 == 1
                odd = np.broadcast_to(rows, X.shape)
                N = lambda x, a=a: (sh(x, -1, a + 1) + sh(x, 1, -a - 1) - sh(x, -1, a) - sh(x, 1, -a)) / 2
                Y = lift(X, odd, N)
                nxt[(cone, 2 * a + 1)] = Y[0::2]
                nxt[(cone, 2 * a)] = Y[1::2]
            else:             # columns split; neighbours (a, -1), (a+1, -1) and mirrors
                cols = np.arange(X.shape[1])[None, :] % 2 == 1
                odd = np.broadcast_to(cols, X.shape)
                N = lambda x, a=a: (sh(x, a + 1, -1) + sh(x, -a - 1, 1) - sh(x, a, -1) - sh(x, -a, 1)) / 2
                Y = lift(X, odd, N)
                nxt[(cone, 2 * a + 1)] = Y[:, 0::2]
                nxt[(cone, 2 * a)] = Y[:, 1::2]
        chans = nxt
    return [chans[(n.cone, n.a)] for n in geo.tree_levels(l)[l]]


@pytest.mark.parametrize("shape,l", [((16, 16), 2), ((32, 32), 3), ((64, 64), 4), ((64, 128), 5)])
def test_operator_form_equals_lifting(shape, l):
    with open(os.path.join(GOLDEN, "lifting_97_published.json")) as f:
        c = json.load(f)
    d = np.random.default_rng(12).uniform(-100, 100, shape)
    ref = _lifting_dfb(d, l, c)
    got = _fwd(d, l)
    for a, b in zip(got, ref):
        assert a.shape == b.shape
        np.testing.assert_allclose(a, b, atol=1e-6)


def _wedge_frequency(k, l, radius, N):
    """FFT-grid frequency (f1, f2) at the angular centre of wedge k."""
    half, q = 2 ** (l - 1), 2 ** (l - 2)
    if k < half:
        a = k - q                       # horizontal: w1/w2 in (a, a+1)/q
        ang = np.arctan((a + 0.5) / q)
        w2, w1 = radius * np.cos(ang), radius * np.sin(ang)
    else:
        a = q - 1 - (k - half)          # vertical: w2/w1 in (a, a+1)/q
        ang = np.arctan((a + 0.5) / q)
        w1, w2 = radius * np.cos(ang), radius * np.sin(ang)
    return round(w1 * N / (2 * np.pi)), round(w2 * N / (2 * np.pi))


@pytest.mark.parametrize("l", [2, 3, 4, 5])
def test_plane_waves_land_in_their_wedge(l):
    """A plane wave at the centre of wedge k puts most energy in subband k.

    The fan filters come from the 9-7 pair and have a wide transition band
    around the cone diagonals, so for the two wedges next to each diagonal
    (l >= 4) the energy may split with the mirror wedge 2^l - 1 - k across
    that diagonal; those two together must still hold most of it.
    """
    N = 256
    n1, n2 = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    nb = 2 ** l
    diag_adjacent = {0, nb // 2 - 1, nb // 2, nb - 1}
    for k in range(nb):
        f1, f2 = _wedge_frequency(k, l, 0.7 * np.pi, N)
        x = np.cos(2 * np.pi * (f1 * n1 + f2 * n2) / N)
        en = np.array([np.sum(s ** 2) for s in _fwd(x, l)])
        if l >= 4 and k in diag_adjacent:
            mirror = nb - 1 - k
            assert en.argmax() in (k, mirror), (k, en.argmax())
            assert en[k] + en[mirror] > 0.85 * en.sum()
            assert en[k] > 0.3 * en.sum()
        else:
            assert en.argmax() == k, (k, en.argmax(), en / en.sum())
            assert en[k] > 0.3 * en.sum()
