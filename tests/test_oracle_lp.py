"""Pins of the LP level (section 2.1 LP; section 3.10: convolutions via FFT, i.e. periodic)."""
import numpy as np
import pytest

from oracle import filters, lp


def _fft_filter2(x, taps):
    """2-D periodic separable filtering computed the paper's way: by FFT."""
    R, C = x.shape
    k = np.zeros((R, C))
    c = len(taps) // 2
    for i, a in enumerate(taps):
        for j, b in enumerate(taps):
            k[(i - c) % R, (j - c) % C] += a * b
    return np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(k)))


@pytest.mark.parametrize("shape", [(16, 16), (24, 40), (64, 32)])
def test_periodic_filtering_matches_fft(shape):
    hbar, gbar = filters.lp_filters()
    x = np.random.default_rng(5).uniform(0, 255, shape)
    for taps in (hbar, gbar):
        np.testing.assert_allclose(lp.filter2(x, taps), _fft_filter2(x, taps), atol=1e-10)


def test_constant_frame_unit_dc():
    hbar, gbar = filters.lp_filters()
    x = np.full((32, 48), 93.25)
    c, d = lp.lp_analysis(x, hbar, gbar)
    np.testing.assert_allclose(c, 93.25, atol=1e-12)
    np.testing.assert_allclose(d, 0.0, atol=1e-12)


def test_half_resolution():
    hbar, gbar = filters.lp_filters()
    c, d = lp.lp_analysis(np.zeros((48, 64)), hbar, gbar)
    assert c.shape == (24, 32) and d.shape == (48, 64)


@pytest.mark.parametrize("shape", [(8, 8), (32, 48), (2, 4)])
def test_lp_perfect_reconstruction(shape):
    hbar, gbar = filters.lp_filters()
    x = np.random.default_rng(6).uniform(0, 255, shape)
    c, d = lp.lp_analysis(x, hbar, gbar)
    np.testing.assert_allclose(lp.lp_synthesis(c, d, hbar, gbar), x, atol=1e-10)


def test_dual_frame_consistency():
    """Synthesis of an arbitrary pair, analysed again, reconstructs the same image.

    Also checks down2 hbar gbar up2 = I, the identity the dual-frame
    reconstruction rests on.
    """
    hbar, gbar = filters.lp_filters()
    rng = np.random.default_rng(7)
    c = rng.standard_normal((8, 8))
    d = rng.standard_normal((16, 16))
    x = lp.lp_synthesis(c, d, hbar, gbar)
    # analysis of the result returns a consistent pair whose synthesis is x again
    c2, d2 = lp.lp_analysis(x, hbar, gbar)
    np.testing.assert_allclose(lp.lp_synthesis(c2, d2, hbar, gbar), x, atol=1e-10)
    # and the lowpass of the reconstruction is the given c (down2 hbar gbar up2 = I)
    np.testing.assert_allclose(lp.down2(lp.filter2(lp.filter2(lp.up2(c), gbar), hbar)), c, atol=1e-12)
