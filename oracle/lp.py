"""Laplacian pyramid (LP) level on a torus.

Paper: section 2.1 (the LP splits an image into a downsampled lowpass and a
full-size bandpass with the missing high frequencies, iterated on the
lowpass), section 3.3 (each level halves the resolution), section 3.10 (the
convolutions are FFT-based, hence periodic).

Reading (unit-DC LP): with hbar = h / sqrt(2) (sum 1) and gbar = g * sqrt(2)
(sum 2), per level, with all indices taken modulo the level size,

  analysis   c = down2(hbar * x)              (separable, kept phase 0)
             d = x - gbar * up2(c)            (up2 inserts zeros at odd indices)
  synthesis  c' = c - down2(hbar * d)         (dual-frame reconstruction)
             x  = d + gbar * up2(c')

Synthesis is exact on unquantised coefficients because down2 hbar gbar up2 is
the identity (biorthogonality of the 9-7 pair).

Variant (not the paper's choice): the original Burt-Adelson reconstruction
skips the correction of c,

  synthesis (BA)  x = d + gbar * up2(c)

and is exact on unquantised coefficients for the same reason (d is then
exactly x - gbar * up2(c)). It differs from the dual-frame reconstruction
only where c and d are not consistent, e.g. after quantisation: an error in d
passes into x unchanged, while the dual frame removes its part that the
lowpass channel sees.

The functions below are generic in the two filters (`lo`, `up`): the forward
transform passes (hbar, gbar). The adjoints of both directions are the same
operations with the filters swapped (see ct.py).
"""
import numpy as np


def conv_periodic(x, taps, axis):
    """y[n] = sum_k taps[k] x[n - k] along `axis`, indices modulo the length.

    `taps` is centred: taps[len // 2] is the coefficient of x[n].
    """
    centre = len(taps) // 2
    y = np.zeros_like(x, dtype=np.float64)
    for idx, t in enumerate(taps):
        k = idx - centre
        y += t * np.roll(x, k, axis=axis)      # roll by k: y[n] gets x[n - k]
    return y


def filter2(x, taps):
    """Separable 2-D periodic filtering with the same 1-D taps on both axes."""
    return conv_periodic(conv_periodic(x, taps, 0), taps, 1)


def down2(x):
    """Keep the samples with both indices even."""
    return x[0::2, 0::2].copy()


def up2(c):
    """Insert zeros at odd row and odd column indices."""
    u = np.zeros((2 * c.shape[0], 2 * c.shape[1]), dtype=np.float64)
    u[0::2, 0::2] = c
    return u


def lp_analysis(x, lo, up):
    """One LP analysis level: returns (c, d)."""
    x = np.asarray(x, dtype=np.float64)
    c = down2(filter2(x, lo))
    d = x - filter2(up2(c), up)
    return c, d


def lp_synthesis(c, d, lo, up):
    """One dual-frame LP synthesis level: returns x."""
    d = np.asarray(d, dtype=np.float64)
    c_corr = np.asarray(c, dtype=np.float64) - down2(filter2(d, lo))
    return d + filter2(up2(c_corr), up)


def lp_synthesis_ba(c, d, up):
    """One Burt-Adelson LP synthesis level: x = d + up * up2(c)."""
    return np.asarray(d, dtype=np.float64) + filter2(up2(np.asarray(c, dtype=np.float64)), up)


def lp_synthesis_ba_adjoint(x, up):
    """Transpose of lp_synthesis_ba: returns (c, d) = (down2(up * x), x).

    filter2 with symmetric taps is self-adjoint and down2 is the transpose of
    up2, so the c part is a lowpass analysis with the synthesis filter; the d
    part is the identity.
    """
    x = np.asarray(x, dtype=np.float64)
    return down2(filter2(x, up)), x.copy()
