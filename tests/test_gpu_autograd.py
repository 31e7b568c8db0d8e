"""GPU tests of the differentiable form: hand-written transposes and autograd.

Workload shape of the differentiation case: 8 planes of 1280x720, J=3,
16/8/4, loss ||S Q_ST(c) - x||^2 + lambda ||c||_1 with step 8 and
lambda = 0.05. The finite-difference check runs on the straight-through
surrogate (quantiser = identity), because finite differences through a
rounding quantiser are not meaningful.
"""
import numpy as np
import pytest
import torch

from oracle import ct as oct
from oracle import geometry as geo
from oracle import matrix
from paper_1510_00561_amd import synth
from tests import clips

pytestmark = pytest.mark.gpu

H5, W5, J5, D5, B5 = 720, 1280, 3, [16, 8, 4], 8
LAM = 0.05


def _plan(H, W, J, dirs, B):
    from paper_1510_00561_amd import ct
    return ct.Plan(H, W, J, dirs, B, "cuda")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).float().cuda()


def test_transposes_equal_explicit_matrix_32x32():
    H = W = 32
    J, dirs = 3, [16, 8, 4]
    R, C = geo.padded_size(H, W, J, dirs)
    M = matrix.forward_matrix(H, W, R, C, J, dirs)
    S = matrix.inverse_matrix(H, W, R, C, J, dirs)
    plan = _plan(H, W, J, dirs, 4)
    rng = np.random.default_rng(41)
    g = rng.standard_normal((4, M.shape[0])).astype(np.float32)
    y = rng.standard_normal((4, H, W)).astype(np.float32)
    fa = plan.forward_adjoint(_dev(g)).cpu().numpy().reshape(4, -1)
    ia = plan.inverse_adjoint(_dev(y)).cpu().numpy()
    for b in range(4):
        want = M.T @ g[b].astype(np.float64)
        assert np.abs(fa[b] - want).max() <= 1e-4 * np.abs(want).max()
        want = S.T @ y[b].ravel().astype(np.float64)
        assert np.abs(ia[b] - want).max() <= 1e-4 * np.abs(want).max()


def test_dot_products_full_size():
    plan = _plan(H5, W5, J5, D5, 2)
    rng = np.random.default_rng(42)
    x = _dev(rng.standard_normal((2, H5, W5)))
    y = _dev(rng.standard_normal((2, plan.ncoef)))
    lhs = (plan.forward(x).double() * y.double()).sum().item()
    rhs = (x.double() * plan.forward_adjoint(y).double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    lhs = (plan.inverse(y).double() * x.double()).sum().item()
    rhs = (y.double() * plan.inverse_adjoint(x).double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


# Worker state of the finite-difference pool: the residual S c - x of every
# plane, set once per worker process.
_FD_RESID = None


def _fd_init(resid):
    global _FD_RESID
    _FD_RESID = resid


def _fd_quadratic(args):
    """Central difference of ||S c - x||^2 along coordinate i of plane b.

    S is linear, so S(c +- h e_i) - x = r +- h S e_i with r = S c - x: the
    loss at both points needs one oracle inverse, of the unit vector."""
    b, i, h, ncoef = args
    e = np.zeros(ncoef)
    e[i] = 1.0
    s = oct.inverse(e, H5, W5, J5, D5)
    r = _FD_RESID[b]
    plus = r + h * s
    minus = r - h * s
    return (float(np.sum(plus * plus)) - float(np.sum(minus * minus))) / (2 * h)


def test_loss_gradient_matches_central_differences():
    """Gradient of ||S c - x||^2 + lambda ||c||_1 (ST surrogate) vs central FD,
    h = 1e-3, at 64 seeded coordinates, eight in each of the 8 planes."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from paper_1510_00561_amd import autograd as ag
    x = np.ascontiguousarray(clips.clip_planes(B5, H5, W5, 5)[0::3])   # the 8 Y planes
    plan = _plan(H5, W5, J5, D5, B5)
    rng = np.random.default_rng(43)
    c_dev = plan.forward(_dev(x)) + 2.0 * torch.from_numpy(
        rng.standard_normal((B5, plan.ncoef)).astype(np.float32)).cuda()
    c = c_dev.clone().requires_grad_(True)
    xd = _dev(x)
    loss = ((ag.ct_inverse(c, plan) - xd) ** 2).sum() + LAM * c.abs().sum()
    loss.backward()
    grad = c.grad.double().cpu().numpy()
    c_np = c_dev.double().cpu().numpy()
    h = 1e-3
    resid = np.stack([oct.inverse(c_np[b], H5, W5, J5, D5) - x[b].astype(np.float64) for b in range(B5)])
    tasks = []
    for b in range(B5):
        cand = np.flatnonzero(np.abs(c_np[b]) > 10 * h)
        for i in rng.choice(cand, size=8, replace=False):
            tasks.append((b, int(i), h, plan.ncoef))
    workers = max(1, min(8, (mp.cpu_count() or 1)))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_fd_init,
                             initargs=(resid,)) as ex:
        quad = list(ex.map(_fd_quadratic, tasks))
    for (b, i, _, _), q in zip(tasks, quad):
        l1 = LAM * (abs(c_np[b, i] + h) - abs(c_np[b, i] - h)) / (2 * h)
        fd = q + l1
        assert abs(grad[b, i] - fd) <= 1e-3 * max(abs(fd), 1.0), (b, i, grad[b, i], fd)


def test_straight_through_quantiser_and_rd_descent():
    from paper_1510_00561_amd import autograd as ag
    H, W, J, dirs, B = 256, 256, 2, [8, 4], 2
    plan = _plan(H, W, J, dirs, B)
    x = _dev(np.stack([synth.luma_edges(H, W, seed=s) for s in (1, 2)]).astype(np.float32))
    steps = torch.full((plan.nsub,), 8.0, device="cuda")
    c = plan.forward(x).clone().requires_grad_(True)
    w = torch.randn_like(c)
    (ag.st_quant(c, steps, plan) * w).sum().backward()
    assert torch.equal(c.grad, w)
    # the rate-distortion loss gradient through the straight-through quantiser
    # is 2 S^T (S Q(c) - x) + lambda sign(c)
    c = plan.forward(x).clone().requires_grad_(True)
    loss = ag.rd_loss(c, x, steps, plan, LAM)
    loss.backward()
    idx, side = plan.quantize(c.detach(), steps)
    resid = plan.inverse(plan.dequantize(idx, steps, side)) - x
    want = 2.0 * plan.inverse_adjoint(resid) + LAM * torch.sign(c.detach())
    assert torch.allclose(c.grad, want, rtol=1e-5, atol=1e-4)
    assert abs(loss.item() - ((resid ** 2).sum() + LAM * c.detach().abs().sum()).item()) <= 1e-5 * loss.item()


def test_forward_autograd_uses_the_forward_transpose():
    from paper_1510_00561_amd import autograd as ag
    H, W, J, dirs, B = 70, 90, 3, [16, 8, 4], 2
    plan = _plan(H, W, J, dirs, B)
    x = torch.randn(B, H, W, device="cuda", requires_grad=True)
    gy = torch.randn(B, plan.ncoef, device="cuda")
    (ag.ct_forward(x, plan) * gy).sum().backward()
    want = plan.forward_adjoint(gy)
    assert torch.allclose(x.grad, want)
