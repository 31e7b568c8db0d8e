"""Pins of the whole contourlet transform (section 2.1 structure, section 3.3 layout)."""
import json
import os

import numpy as np
import pytest

from oracle import ct, matrix
from oracle import geometry as geo


@pytest.mark.parametrize("H,W,J,dirs", [
    (16, 16, 2, [8, 4]),
    (64, 64, 2, [8, 4]),
    (40, 56, 2, [4, 4]),          # unpadded (multiples of 4)
    (72, 96, 3, [16, 8, 4]),      # unpadded (multiples of 8)
    (70, 90, 3, [16, 8, 4]),      # padded to 72 x 96
    (64, 64, 1, [64]),
    (33, 65, 1, [4]),
])
def test_perfect_reconstruction(H, W, J, dirs):
    x = np.random.default_rng(21).uniform(0, 255, (H, W))
    v = ct.forward(x, J, dirs)
    assert v.size == geo.ncoef(H, W, J, dirs)
    np.testing.assert_allclose(ct.inverse(v, H, W, J, dirs), x, atol=1e-10)


def test_constant_frame():
    H, W, J, dirs = 48, 80, 3, [16, 8, 4]
    v = ct.forward(np.full((H, W), 117.0), J, dirs)
    n_low = geo.subband_table(H, W, J, dirs)[0].size
    np.testing.assert_allclose(v[:n_low], 117.0, atol=1e-12)
    np.testing.assert_allclose(v[n_low:], 0.0, atol=1e-11)


def test_linearity():
    H, W, J, dirs = 32, 48, 2, [8, 4]
    rng = np.random.default_rng(22)
    x, y = rng.standard_normal((2, H, W))
    a, b = 2.5, -0.75
    lhs = ct.forward(a * x + b * y, J, dirs)
    rhs = a * ct.forward(x, J, dirs) + b * ct.forward(y, J, dirs)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(rhs).max())


def test_shift_covariance():
    """Shifting the frame by (2^e, 2^e) cyclically shifts every subband array.

    Subband k of level j samples the level image on o + diag(s1, s2) Z^2 and
    the level image is the frame at 2^(j-1) times coarser resolution, so the
    subband shifts by 2^e / (2^(j-1) s1) rows and 2^e / (2^(j-1) s2) columns.
    """
    H, W, J, dirs = 64, 64, 2, [16, 4]
    e = geo.pad_exponent(J, dirs)
    x = np.random.default_rng(23).standard_normal((H, W))
    xs = np.roll(x, (1 << e, 1 << e), axis=(0, 1))
    table = geo.subband_table(H, W, J, dirs)
    low, subs = ct.unpack(ct.forward(x, J, dirs), table, J)
    low_s, subs_s = ct.unpack(ct.forward(xs, J, dirs), table, J)
    np.testing.assert_allclose(low_s, np.roll(low, ((1 << e) >> J,) * 2, axis=(0, 1)), atol=1e-12)
    for sb in table[1:]:
        scale = 1 << (sb.level - 1)
        dr = (1 << e) // (scale * sb.s1)
        dc = (1 << e) // (scale * sb.s2)
        got = subs_s[sb.level - 1][sb.k]
        want = np.roll(subs[sb.level - 1][sb.k], (dr, dc), axis=(0, 1))
        np.testing.assert_allclose(got, want, atol=1e-11)


@pytest.fixture(scope="module")
def c1_matrices():
    H = W = 16
    J, dirs = 2, [8, 4]
    R, C = geo.padded_size(H, W, J, dirs)
    return (H, W, J, dirs), matrix.forward_matrix(H, W, R, C, J, dirs), matrix.inverse_matrix(H, W, R, C, J, dirs)


def test_explicit_matrix_forward(c1_matrices):
    (H, W, J, dirs), M, _ = c1_matrices
    n = H * W
    fast = np.stack([ct.forward(np.eye(n)[i].reshape(H, W), J, dirs) for i in range(n)], 1)
    np.testing.assert_allclose(fast, M, atol=1e-12)


def test_explicit_matrix_inverse_and_frame(c1_matrices):
    (H, W, J, dirs), M, S = c1_matrices
    nc = M.shape[0]
    fast = np.stack([ct.inverse(np.eye(nc)[i], H, W, J, dirs).ravel() for i in range(nc)], 1)
    np.testing.assert_allclose(fast, S, atol=1e-12)
    np.testing.assert_allclose(S @ M, np.eye(H * W), atol=1e-12)
    np.testing.assert_allclose(M @ S @ M, M, atol=1e-12)
    sv = np.linalg.svd(M, compute_uv=False)
    assert sv.max() / sv.min() > 1.5, "frame should not be tight"
    # forward^T is not the inverse for this frame
    assert np.abs(S - M.T).max() > 1e-2


def test_adjoint_dot_products():
    H, W, J, dirs = 40, 56, 2, [8, 4]
    rng = np.random.default_rng(24)
    x = rng.standard_normal((H, W))
    y = rng.standard_normal(geo.ncoef(H, W, J, dirs))
    lhs = np.dot(ct.forward(x, J, dirs), y)
    rhs = np.dot(x.ravel(), ct.forward_adjoint(y, H, W, J, dirs).ravel())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    lhs = np.dot(ct.inverse(y, H, W, J, dirs).ravel(), x.ravel())
    rhs = np.dot(y, ct.inverse_adjoint(x, H, W, J, dirs))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_adjoints_equal_explicit_transpose_32():
    """On 32x32 crops with the differentiation geometry (J=3, 16/8/4)."""
    H = W = 32
    J, dirs = 3, [16, 8, 4]
    R, C = geo.padded_size(H, W, J, dirs)
    M = matrix.forward_matrix(H, W, R, C, J, dirs)
    S = matrix.inverse_matrix(H, W, R, C, J, dirs)
    rng = np.random.default_rng(25)
    for _ in range(3):
        g = rng.standard_normal(M.shape[0])
        np.testing.assert_allclose(ct.forward_adjoint(g, H, W, J, dirs).ravel(), M.T @ g, atol=1e-11)
        y = rng.standard_normal(H * W)
        np.testing.assert_allclose(ct.inverse_adjoint(y.reshape(H, W), H, W, J, dirs), S.T @ y, atol=1e-11)


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_padding_worked_example():
    """The mirror extension on a hand-worked 3 x 4 -> 5 x 7 example."""
    with open(os.path.join(GOLDEN, "pad_worked.json")) as f:
        g = json.load(f)
    x = np.array(g["frame"], dtype=np.float64)
    R, C = g["padded_rc"]
    np.testing.assert_array_equal(ct._pad(x, R, C), np.array(g["padded"], dtype=np.float64))
    np.testing.assert_array_equal(matrix.pad_matrix(*x.shape, R, C) @ x.ravel(),
                                  np.array(g["padded"], dtype=np.float64).ravel())


def test_pad_adjoint_is_transpose():
    H, W, R, C = 13, 11, 16, 16
    P = matrix.pad_matrix(H, W, R, C)
    y = np.random.default_rng(26).standard_normal((R, C))
    np.testing.assert_allclose(ct._pad_adjoint(y, H, W).ravel(), P.T @ y.ravel(), atol=1e-13)


@pytest.fixture(scope="module")
def padded_matrices():
    """14 x 18, J = 2, dirs 8/4: padded to 16 x 20 (rows and columns)."""
    H, W, J, dirs = 14, 18, 2, [8, 4]
    R, C = geo.padded_size(H, W, J, dirs)
    assert (R, C) == (16, 20)
    return (H, W, J, dirs), matrix.forward_matrix(H, W, R, C, J, dirs), matrix.inverse_matrix(H, W, R, C, J, dirs)


def test_explicit_matrix_padded(padded_matrices):
    """The array path equals the stage-by-stage matrices on a padded geometry,
    so the padding rule (and the crop) are fixed by an independent route."""
    (H, W, J, dirs), M, S = padded_matrices
    n = H * W
    fast = np.stack([ct.forward(np.eye(n)[i].reshape(H, W), J, dirs) for i in range(n)], 1)
    np.testing.assert_allclose(fast, M, atol=1e-12)
    nc = M.shape[0]
    rng = np.random.default_rng(27)
    for _ in range(3):
        v = rng.standard_normal(nc)
        np.testing.assert_allclose(ct.inverse(v, H, W, J, dirs).ravel(), S @ v, atol=1e-11)
    np.testing.assert_allclose(S @ M, np.eye(n), atol=1e-11)


def test_adjoints_explicit_transpose_padded(padded_matrices):
    (H, W, J, dirs), M, S = padded_matrices
    rng = np.random.default_rng(28)
    for _ in range(3):
        g = rng.standard_normal(M.shape[0])
        np.testing.assert_allclose(ct.forward_adjoint(g, H, W, J, dirs).ravel(), M.T @ g, atol=1e-11)
        y = rng.standard_normal(H * W)
        np.testing.assert_allclose(ct.inverse_adjoint(y.reshape(H, W), H, W, J, dirs), S.T @ y, atol=1e-11)


def test_adjoint_dot_products_padded():
    H, W, J, dirs = 70, 90, 3, [16, 8, 4]
    rng = np.random.default_rng(29)
    x = rng.standard_normal((H, W))
    y = rng.standard_normal(geo.ncoef(H, W, J, dirs))
    lhs = np.dot(ct.forward(x, J, dirs), y)
    rhs = np.dot(x.ravel(), ct.forward_adjoint(y, H, W, J, dirs).ravel())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    lhs = np.dot(ct.inverse(y, H, W, J, dirs).ravel(), x.ravel())
    rhs = np.dot(y, ct.inverse_adjoint(x, H, W, J, dirs))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
