"""Pins of the closed-form 9-7 pair (section 2.1 names the Cohen-Daubechies 9-7 filters)."""
import json
import os

import numpy as np

from oracle import filters

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_taps_match_published_values():
    ref = _load("cdf97_published.json")
    h, g = filters.cdf97_taps()
    assert len(h) == 9 and len(g) == 7
    np.testing.assert_allclose(h[4:], ref["analysis_lowpass_h0_to_h4"], atol=ref["tolerance"])
    np.testing.assert_allclose(g[3:], ref["synthesis_lowpass_g0_to_g3"], atol=ref["tolerance"])
    # symmetric (zero phase)
    np.testing.assert_array_equal(h, h[::-1])
    np.testing.assert_array_equal(g, g[::-1])


def test_halfband_identity():
    # h(w) g(w) + h(w + pi) g(w + pi) = 2 on a dense grid
    p, q = filters.cdf97_polynomials()
    t = np.cos(np.linspace(0, np.pi, 1001))
    val = np.polyval(p[::-1], t) * np.polyval(q[::-1], t) + np.polyval(p[::-1], -t) * np.polyval(q[::-1], -t)
    np.testing.assert_allclose(val, 2.0, atol=1e-14)


def test_biorthogonality():
    # sum_n h[n] g[n - 2k] = delta_k
    h, g = filters.cdf97_taps()
    for k in range(-4, 5):
        s = 0.0
        for n in range(-4, 5):
            m = n - 2 * k
            if -3 <= m <= 3:
                s += h[n + 4] * g[m + 3]
        assert abs(s - (1.0 if k == 0 else 0.0)) < 1e-15


def test_four_vanishing_moments_at_pi():
    h, g = filters.cdf97_taps()
    for taps in (h, g):
        n = np.arange(len(taps)) - len(taps) // 2
        for k in range(4):
            assert abs(np.sum((-1.0) ** n * n ** k * taps)) < 1e-13
    # and sum sqrt(2) each
    assert abs(h.sum() - np.sqrt(2)) < 1e-15 and abs(g.sum() - np.sqrt(2)) < 1e-15


def test_lifting_factorisation_reproduces_the_pair():
    """Published lifting constants (an independent algorithm) give E p(T), O q(-T).

    1-D torus of length 32, T = (S + S^-1)/2. Lifting: odd += alpha (left+right
    even), even += beta (...), odd += gamma, even += delta, even *= zeta,
    odd /= zeta.
    """
    ref = _load("lifting_97_published.json")
    p, q = filters.cdf97_polynomials()
    N = 32
    x = np.random.default_rng(3).standard_normal(N)

    def T(v):
        return (np.roll(v, 1) + np.roll(v, -1)) / 2

    def poly(c, v, op):
        y = c[-1] * v
        for a in c[-2::-1]:
            y = op(y) + a * v
        return y

    even = np.arange(N) % 2 == 0
    want = np.where(even, poly(p, x, T), poly(q, x, lambda v: -T(v)))
    z = x.copy()
    nb = lambda v: np.roll(v, 1) + np.roll(v, -1)
    for coef, upd in ((ref["alpha"], ~even), (ref["beta"], even), (ref["gamma"], ~even), (ref["delta"], even)):
        z = z + np.where(upd, coef * nb(np.where(upd, 0.0, z)), 0.0)
    z = np.where(even, z * ref["zeta"], z / ref["zeta"])
    np.testing.assert_allclose(z, want, atol=ref["tolerance"] * 10 * np.abs(x).max())
