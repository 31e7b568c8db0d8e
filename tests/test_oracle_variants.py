"""Pins of the variant filters and reconstruction (not the paper's choices).

The paper (section 2.1) uses the 9-7 pair and a Laplacian pyramid whose
reconstruction it does not spell out; the oracle's default is the dual-frame
synthesis. Two variants stand beside them:
  * the LeGall 5/3 pair (filters.legall53_polynomials) for the LP and the
    fan filters of the DFB;
  * the Burt-Adelson LP reconstruction x = d + gbar * up2(c)
    (lp.lp_synthesis_ba).
Each is pinned by values or properties that a mistake in it would break:
textbook taps, zeros at pi, the halfband identity, perfect reconstruction,
the explicit matrices of matrix.py (written without the array code), the
closed form of how an error in d reaches the output, and the adjoints.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly

from oracle import ct, filters, lp, matrix
from oracle import geometry as geo

VARIANTS = [("97", "dual"), ("97", "ba"), ("53", "dual"), ("53", "ba")]


def test_legall53_taps_are_the_textbook_pair():
    """Unit-DC LP taps of the 5/3 pair: analysis (-1, 2, 6, 2, -1)/8 and
    synthesis (1, 2, 1)/2 (the reversible pair of lossless wavelet coding),
    here with the synthesis filter scaled to sum 2 like gbar."""
    hbar, gbar = filters.lp_filters("53")
    np.testing.assert_allclose(hbar, np.array([-1, 2, 6, 2, -1]) / 8.0, atol=1e-15)
    np.testing.assert_allclose(gbar, np.array([1, 2, 1]) / 2.0, atol=1e-15)


@pytest.mark.parametrize("kind,zeros", [("53", (2, 2)), ("97", (4, 4))])
def test_zeros_at_pi_and_halfband(kind, zeros):
    """h(w) and g(w) vanish at w = pi (t = -1) to the order of their
    cos^2(w/2) factors (two zeros per factor in w, one per factor in t), and
    p(t) q(t) + p(-t) q(-t) = 2, the condition for perfect reconstruction."""
    p, q = filters.polynomials(kind)
    for poly, nz in zip((p, q), zeros):
        d = np.asarray(poly, dtype=np.float64)
        for _ in range(nz // 2):
            assert abs(npoly.polyval(-1.0, d)) < 1e-12
            d = npoly.polyder(d)
        assert abs(npoly.polyval(-1.0, d)) > 1e-3
        assert abs(npoly.polyval(1.0, poly) - np.sqrt(2.0)) < 1e-14
    s = npoly.polyadd(npoly.polymul(p, q),
                      npoly.polymul(filters.negate_argument(p), filters.negate_argument(q)))
    s = np.trim_zeros(np.round(s, 13), "b")
    np.testing.assert_allclose(s, [2.0], atol=1e-13)


@pytest.mark.parametrize("kind,recon", VARIANTS)
@pytest.mark.parametrize("H,W,J,dirs", [
    (64, 64, 2, [8, 4]),
    (70, 90, 3, [16, 8, 4]),      # padded to 72 x 96
    (33, 65, 1, [32]),
])
def test_perfect_reconstruction(kind, recon, H, W, J, dirs):
    x = np.random.default_rng(31).uniform(0, 255, (H, W))
    v = ct.forward(x, J, dirs, filters=kind)
    np.testing.assert_allclose(ct.inverse(v, H, W, J, dirs, filters=kind, recon=recon), x, atol=1e-10)


def test_53_differs_from_97():
    H, W, J, dirs = 32, 32, 2, [8, 4]
    x = np.random.default_rng(32).uniform(0, 255, (H, W))
    assert np.abs(ct.forward(x, J, dirs, filters="53") - ct.forward(x, J, dirs)).max() > 1.0


def test_constant_frame_53():
    H, W, J, dirs = 48, 80, 3, [16, 8, 4]
    v = ct.forward(np.full((H, W), 117.0), J, dirs, filters="53")
    n_low = geo.subband_table(H, W, J, dirs)[0].size
    np.testing.assert_allclose(v[:n_low], 117.0, atol=1e-12)
    np.testing.assert_allclose(v[n_low:], 0.0, atol=1e-11)


def test_ba_passes_an_error_in_d_unchanged():
    """One LP level: BA maps (c, d + e) to x + e exactly; the dual frame maps
    it to x + e - gbar * up2(down2(hbar * e)), i.e. removes the part of e that
    the lowpass channel sees."""
    rng = np.random.default_rng(33)
    hbar, gbar = filters.lp_filters("97")
    x = rng.standard_normal((32, 48))
    c, d = lp.lp_analysis(x, hbar, gbar)
    e = rng.standard_normal(d.shape)
    np.testing.assert_allclose(lp.lp_synthesis_ba(c, d + e, gbar), x + e, atol=1e-12)
    seen = lp.filter2(lp.up2(lp.down2(lp.filter2(e, hbar))), gbar)
    np.testing.assert_allclose(lp.lp_synthesis(c, d + e, hbar, gbar), x + e - seen, atol=1e-12)
    assert np.abs(seen).max() > 0.1


def test_ba_and_dual_agree_on_consistent_coefficients_only():
    H, W, J, dirs = 40, 56, 2, [8, 4]
    rng = np.random.default_rng(34)
    v = ct.forward(rng.uniform(0, 255, (H, W)), J, dirs)
    a = ct.inverse(v, H, W, J, dirs, recon="ba")
    b = ct.inverse(v, H, W, J, dirs, recon="dual")
    np.testing.assert_allclose(a, b, atol=1e-10)
    noisy = v + rng.uniform(-4, 4, v.shape)
    a = ct.inverse(noisy, H, W, J, dirs, recon="ba")
    b = ct.inverse(noisy, H, W, J, dirs, recon="dual")
    assert np.abs(a - b).max() > 0.1


@pytest.fixture(scope="module", params=[("53", "dual"), ("53", "ba"), ("97", "ba")])
def variant_matrices(request):
    kind, recon = request.param
    H, W = 14, 18                 # padded to 16 x 20: the mirror rows and columns are in the matrices
    J, dirs = 2, [8, 4]
    R, C = geo.padded_size(H, W, J, dirs)
    assert (R, C) != (H, W)
    M = matrix.forward_matrix(H, W, R, C, J, dirs, kind)
    S = matrix.inverse_matrix(H, W, R, C, J, dirs, kind, recon)
    return kind, recon, (H, W, J, dirs), M, S


def test_explicit_matrices(variant_matrices):
    kind, recon, (H, W, J, dirs), M, S = variant_matrices
    n = H * W
    fwd = np.stack([ct.forward(np.eye(n)[i].reshape(H, W), J, dirs, filters=kind) for i in range(n)], 1)
    np.testing.assert_allclose(fwd, M, atol=1e-12)
    nc = M.shape[0]
    cols = [0, 1, 7, nc // 3, nc // 2, nc - 5, nc - 1]
    for i in cols:
        got = ct.inverse(np.eye(nc)[i], H, W, J, dirs, filters=kind, recon=recon).ravel()
        np.testing.assert_allclose(got, S[:, i], atol=1e-12)
    np.testing.assert_allclose(S @ M, np.eye(n), atol=1e-11)


def test_adjoints_equal_explicit_transposes(variant_matrices):
    kind, recon, (H, W, J, dirs), M, S = variant_matrices
    rng = np.random.default_rng(35)
    g = rng.standard_normal(M.shape[0])
    np.testing.assert_allclose(ct.forward_adjoint(g, H, W, J, dirs, filters=kind).ravel(), M.T @ g, atol=1e-11)
    y = rng.standard_normal(H * W)
    np.testing.assert_allclose(ct.inverse_adjoint(y.reshape(H, W), H, W, J, dirs, filters=kind, recon=recon),
                               S.T @ y, atol=1e-11)


@pytest.mark.parametrize("kind,recon", VARIANTS)
def test_adjoint_dot_products(kind, recon):
    H, W, J, dirs = 36, 52, 2, [8, 16]
    rng = np.random.default_rng(36)
    x = rng.standard_normal((H, W))
    y = rng.standard_normal(geo.ncoef(H, W, J, dirs))
    lhs = np.dot(ct.inverse(y, H, W, J, dirs, filters=kind, recon=recon).ravel(), x.ravel())
    rhs = np.dot(y, ct.inverse_adjoint(x, H, W, J, dirs, filters=kind, recon=recon))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    lhs = np.dot(ct.forward(x, J, dirs, filters=kind), y)
    rhs = np.dot(x.ravel(), ct.forward_adjoint(y, H, W, J, dirs, filters=kind).ravel())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
