"""Cohen-Daubechies 9-7 biorthogonal filter pair in closed form.

Paper: section 2.1 states that the LP and the DFB both use the Cohen and
Daubechies 9-7 filters. Neither the taps nor their normalisation are printed,
so they are derived here from the defining construction of the pair:

  * let y = sin^2(w/2) = (1 - cos w)/2 and Q(y) = 1 + 4y + 10y^2 + 20y^3, the
    remainder polynomial of the Daubechies halfband product with four zeros
    at w = pi (p = 4);
  * Q has one real root y_r and a complex-conjugate pair y_1, conj(y_1);
  * analysis lowpass   h(w) = c_h cos^4(w/2) (y - y_1)(y - conj y_1)  (9 taps)
  * synthesis lowpass  g(w) = c_g cos^4(w/2) (y - y_r)                (7 taps)
  * both are zero-phase and normalised so that h(0) = g(0) = sqrt(2).

Then h(w) g(w) + h(w + pi) g(w + pi) = 2 (the halfband identity), which is
what makes the LP invertible and the fan filter bank perfectly
reconstructing.

Both filters are even in w, hence polynomials in t = cos w:
  p(t) = h(w), degree 4;   q(t) = g(w), degree 3.
The DFB uses p and q directly as polynomials of the fan kernel; the LP uses
the taps obtained by t = (z + 1/z)/2.
"""
import numpy as np
from numpy.polynomial import polynomial as npoly


def _remainder_roots():
    """Roots of Q(y) = 1 + 4y + 10y^2 + 20y^3: (real root, upper complex root)."""
    roots = np.roots([20.0, 10.0, 4.0, 1.0])
    real = roots[np.argmin(np.abs(roots.imag))].real
    upper = roots[np.argmax(roots.imag)]
    return float(real), complex(upper)


def cdf97_polynomials():
    """Return (p, q): coefficient arrays (lowest degree first) in t = cos(w).

    p(t) = h(w) is the 9-tap analysis lowpass, q(t) = g(w) the 7-tap
    synthesis lowpass, both with value sqrt(2) at t = 1 (w = 0).
    """
    y_r, y_1 = _remainder_roots()
    half_plus = np.array([0.5, 0.5])              # cos^2(w/2) = (1 + t)/2

    def y_minus(root):                            # y - root, y = (1 - t)/2
        return np.array([0.5 - root, -0.5])

    cos4 = npoly.polymul(half_plus, half_plus)
    p = npoly.polymul(cos4, npoly.polymul(y_minus(y_1), y_minus(np.conj(y_1))))
    q = npoly.polymul(cos4, y_minus(y_r))
    p = np.real_if_close(p).astype(np.float64)
    q = np.real_if_close(q).astype(np.float64)
    p = p * (np.sqrt(2.0) / npoly.polyval(1.0, p))
    q = q * (np.sqrt(2.0) / npoly.polyval(1.0, q))
    return p, q


def poly_to_taps(poly):
    """Symmetric taps f[-n..n] of the Laurent polynomial f(z) = P((z + 1/z)/2).

    Expands t^k = ((z + 1/z)/2)^k term by term; index n of the result is the
    centre tap.
    """
    n = len(poly) - 1
    taps = np.zeros(2 * n + 1)
    power = np.zeros(2 * n + 1)
    power[n] = 1.0                                # t^0
    for coef in poly:
        taps += coef * power
        nxt = np.zeros_like(power)
        nxt[1:] += 0.5 * power[:-1]
        nxt[:-1] += 0.5 * power[1:]
        power = nxt
    return taps


def cdf97_taps():
    """Return (h, g): 9 analysis-lowpass taps h[-4..4], 7 synthesis taps g[-3..3].

    Normalised to sum sqrt(2) each (the unit-energy-style normalisation).
    """
    p, q = cdf97_polynomials()
    return poly_to_taps(p), poly_to_taps(q)


def legall53_polynomials():
    """Return (p, q) of the LeGall 5/3 pair, lowest degree first, in t = cos(w).

    A variant filter pair (not the paper's): the same construction as the
    9-7 pair with two zeros at w = pi on each side instead of four. The
    Daubechies halfband product with two zeros at pi has the remainder
    polynomial Q(y) = 1 + 2y; the synthesis lowpass takes cos^2(w/2) alone
    and the analysis lowpass cos^2(w/2) Q(y), both normalised to sqrt(2) at
    t = 1:
      p(t) = h(w), degree 2 (5 taps);   q(t) = g(w), degree 1 (3 taps).
    """
    half_plus = np.array([0.5, 0.5])              # cos^2(w/2) = (1 + t)/2
    remainder = np.array([2.0, -1.0])             # 1 + 2y with y = (1 - t)/2
    p = npoly.polymul(half_plus, remainder)
    q = half_plus.copy()
    p = p * (np.sqrt(2.0) / npoly.polyval(1.0, p))
    q = q * (np.sqrt(2.0) / npoly.polyval(1.0, q))
    return p, q


FILTERS = {'97': cdf97_polynomials, '53': legall53_polynomials}


def polynomials(kind='97'):
    """(p, q) of filter pair `kind`: '97' (the paper's 9-7) or '53' (LeGall 5/3)."""
    return FILTERS[kind]()


def lp_filters(kind='97'):
    """LP filters of the unit-DC reading (O-3 of the contourlet reading).

    hbar = h / sqrt(2) sums to 1 (the 2-D lowpass keeps the pixel scale),
    gbar = g * sqrt(2) sums to 2 (so that gbar applied to an upsampled
    constant returns the constant). Both are centred: index len//2 is tap 0.
    """
    p, q = polynomials(kind)
    return poly_to_taps(p) / np.sqrt(2.0), poly_to_taps(q) * np.sqrt(2.0)


def negate_argument(poly):
    """Coefficients of f(-t) given those of f(t)."""
    signs = np.array([(-1.0) ** k for k in range(len(poly))])
    return np.asarray(poly) * signs
