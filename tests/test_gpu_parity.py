"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: FP32 coefficients and reconstructions agree with the FP64 oracle
to max-abs 1e-3 on the 0-255 pixel scale. Quantiser indices and side info
are bit-exact against the oracle's FP32 quantiser given the same FP32
coefficients (the oracle's own coefficients rounded to FP32). Dequantised
values are bit-exact against the oracle's FP32 dequantiser.
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import ct as oct
from oracle import geometry as geo
from oracle import quant as oq
from paper_1510_00561_amd import synth
from tests import clips

pytestmark = pytest.mark.gpu

TOL = 1e-3


def _plan(H, W, J, dirs, B):
    from paper_1510_00561_amd import ct
    return ct.Plan(H, W, J, dirs, B, "cuda")


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _frames(name, H, W, B):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name == "c1":
        return synth.luma_edges(H, W)[None].astype(np.float32)
    if name in ("c2", "c3", "c5"):
        n_frames = max(1, B // 3)
        planes = clips.clip_planes(n_frames, H, W, {"c2": 2, "c3": 3, "c5": 5}[name])
        return planes[:B]
    return rng.uniform(0, 255, (B, H, W)).astype(np.float32)


CASES = [
    ("c1", 256, 256, 2, [8, 4], 1),
    ("tiny", 16, 16, 2, [8, 4], 2),
    ("ragged", 70, 90, 3, [16, 8, 4], 2),
    ("c2", 480, 640, 3, [16, 8, 4], 3),
    ("dirs64", 128, 128, 1, [64], 1),
    ("mixed", 64, 96, 2, [4, 32], 2),
    ("deep6", 192, 256, 6, [8, 8, 4, 4, 4, 4], 1),
    ("c5", 720, 1280, 3, [16, 8, 4], 1),
    # odd coefficient count (5x5 lowpass): every other plane's indices start
    # at an odd element
    ("oddlow", 40, 40, 3, [8, 4, 4], 3),
    # smallest frames: a one-level split of 2-row parents, a two-level split
    # of 4x4 parents
    ("min8", 4, 4, 1, [8], 2),
    ("min16", 8, 8, 1, [16], 2),
    # channels narrower than a strip, rows wider than two strips
    ("wide", 24, 200, 2, [16, 4], 2),
]


def _show(name, **kw):
    print(f"[parity] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("name,H,W,J,dirs,B", CASES, ids=[c[0] for c in CASES])
def test_forward_inverse_parity(name, H, W, J, dirs, B):
    _show(name, H=H, W=W, J=J, dirs=dirs, B=B)
    x = _frames(name, H, W, B)
    plan = _plan(H, W, J, dirs, B)
    coef = plan.forward(_dev(x))
    rec = plan.inverse(coef)
    torch.cuda.synchronize()
    coef_h = coef.cpu().numpy()
    rec_h = rec.cpu().numpy()
    for b in range(B):
        ref = oct.forward(x[b].astype(np.float64), J, dirs)
        err = np.abs(coef_h[b] - ref).max()
        assert err <= TOL, f"plane {b}: forward max abs err {err}"
        # the GPU round trip restores the input
        assert np.abs(rec_h[b] - x[b]).max() <= TOL
    # inverse of the oracle's coefficients (as FP32) against the oracle inverse
    ref_c32 = np.stack([oct.forward(x[b].astype(np.float64), J, dirs) for b in range(B)]).astype(np.float32)
    rec2 = plan.inverse(_dev(ref_c32)).cpu().numpy()
    for b in range(B):
        want = oct.inverse(ref_c32[b].astype(np.float64), H, W, J, dirs)
        assert np.abs(rec2[b] - want).max() <= TOL


QCASES = CASES[:5] + [c for c in CASES if c[0] in ("oddlow", "min8", "wide")]


@pytest.mark.parametrize("name,H,W,J,dirs,B", QCASES, ids=[c[0] for c in QCASES])
def test_quantiser_bit_exact(name, H, W, J, dirs, B):
    _show(name, H=H, W=W, J=J, dirs=dirs, B=B)
    x = _frames(name, H, W, B)
    plan = _plan(H, W, J, dirs, B)
    table = geo.subband_table(H, W, J, dirs)
    c32 = np.stack([oct.forward(x[b].astype(np.float64), J, dirs) for b in range(B)]).astype(np.float32)
    steps = np.random.default_rng(7).integers(1, 65, size=(B, len(table))).astype(np.float32)
    idx, side = plan.quantize(_dev(c32), _dev(steps))
    deq = plan.dequantize(idx, _dev(steps), side)
    torch.cuda.synchronize()
    idx_h, side_h, deq_h = idx.cpu().numpy(), side.cpu().numpy(), deq.cpu().numpy()
    for b in range(B):
        q_ref, s_ref = oq.quantize32(c32[b], steps[b], table)
        np.testing.assert_array_equal(idx_h[b], q_ref)
        assert side_h[b, 0] == s_ref[0] and side_h[b, 1] == s_ref[1]
        d_ref = oq.dequantize32(q_ref, steps[b], s_ref, table)
        np.testing.assert_array_equal(deq_h[b], d_ref)
    # arrays 4 bytes off a 16-byte boundary take the per-element path
    n = B * plan.ncoef
    cbuf = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    cbuf[1:] = _dev(c32).reshape(-1)
    ibuf = torch.zeros(n + 1, dtype=torch.int16, device="cuda")
    dbuf = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    idx_m, side_m = plan.quantize(cbuf[1:].view(B, plan.ncoef), _dev(steps), idx=ibuf[1:].view(B, plan.ncoef))
    deq_m = plan.dequantize(idx_m, _dev(steps), side_m, out=dbuf[1:].view(B, plan.ncoef))
    assert torch.equal(idx_m.cpu(), idx.cpu()) and torch.equal(side_m.cpu(), side.cpu())
    assert torch.equal(deq_m.cpu(), deq.cpu())
    # shared step row (stride 0)
    idx2, _ = plan.quantize(_dev(c32), _dev(steps[0]))
    idx2_h = idx2.cpu().numpy()
    for b in range(B):
        np.testing.assert_array_equal(idx2_h[b], oq.quantize32(c32[b], steps[0], table)[0])


def test_quantiser_ties_and_limits():
    H, W, J, dirs = 16, 16, 1, [4]
    table = geo.subband_table(H, W, J, dirs)
    n = table[-1].offset + table[-1].size
    c = np.zeros((2, n), np.float32)
    c[0, :table[0].size] = 42.0                      # constant lowpass -> s = 0
    vals = np.array([0.5, 1.5, 2.5, -0.5, -2.5, 0.49999997, 1e9, -1e9, 3.75,
                     np.inf, -np.inf, np.nan, -0.0, 1e-45, 32766.5, -32767.5, 8388607.5, -8388607.5,
                     0.50000006, -1.4999999], np.float32)
    c[:, table[1].offset:table[1].offset + len(vals)] = vals
    c[1, :table[0].size] = np.linspace(-3, 7, table[0].size, dtype=np.float32)
    steps = np.ones(len(table), np.float32)
    plan = _plan(H, W, J, dirs, 2)
    idx, side = plan.quantize(_dev(c), _dev(steps))
    idx_h, side_h = idx.cpu().numpy(), side.cpu().numpy()
    for b in range(2):
        q_ref, s_ref = oq.quantize32(c[b], steps, table)
        np.testing.assert_array_equal(idx_h[b], q_ref)
        assert tuple(side_h[b]) == tuple(np.float32(v) for v in s_ref)
    assert np.all(idx_h[0, :table[0].size] == 0)
    assert list(idx_h[0, table[1].offset:table[1].offset + len(vals)]) == [
        1, 2, 3, -1, -3, 0, 32767, -32768, 4,
        32767, -32768, 0, 0, 0, 32767, -32768, 32767, -32768, 1, -1]


def _near_half_integers(table, steps, B, seed):
    """Coefficients at and a few float32 steps around (k + 1/2) * step for every
    directional subband, k up to the int16 range: the values whose index
    depends on the quotient's last bit and on the direction of the tie rule."""
    rng = np.random.default_rng(seed)
    n = table[-1].offset + table[-1].size
    c = rng.uniform(-300, 300, (B, n)).astype(np.float32)
    for s, sb in enumerate(table):
        if s == 0:
            continue
        m = sb.size
        k = rng.integers(-32800, 32800, size=(B, m)).astype(np.float64)
        k[:, : m // 2] = rng.integers(-40, 40, size=(B, m // 2))
        base = ((k + 0.5) * np.float64(steps[s])).astype(np.float32)
        ulps = rng.integers(-3, 4, size=(B, m))
        v = base.copy()
        for _ in range(3):
            up = ulps > 0
            down = ulps < 0
            v = np.where(up, np.nextafter(v, np.float32(np.inf)), v)
            v = np.where(down, np.nextafter(v, np.float32(-np.inf)), v)
            ulps = ulps - np.sign(ulps)
        c[:, sb.offset:sb.offset + m] = v
    return c


@pytest.mark.parametrize("case", ["integer", "fractional", "extreme"])
def test_quantiser_near_half_integers(case):
    H, W, J, dirs, B = 64, 96, 2, [4, 32], 3
    table = geo.subband_table(H, W, J, dirs)
    rng = np.random.default_rng({"integer": 1, "fractional": 2, "extreme": 3}[case])
    if case == "integer":
        steps = rng.integers(3, 65, size=len(table)).astype(np.float32)
    elif case == "fractional":
        steps = rng.choice(np.array([0.1, 0.37, 7.5, 1e-3, 13.25, 0.0625], np.float32), size=len(table))
    else:   # steps near the float32 exponent limits
        steps = rng.choice(np.array([2.0 ** -101, 2.0 ** 101, 3.0, 2.0 ** -99], np.float32), size=len(table))
    c = _near_half_integers(table, steps, B, 7)
    plan = _plan(H, W, J, dirs, B)
    idx, side = plan.quantize(_dev(c), _dev(steps))
    idx_h = idx.cpu().numpy()
    for b in range(B):
        q_ref, _ = oq.quantize32(c[b], steps, table)
        np.testing.assert_array_equal(idx_h[b], q_ref)


def _tricky_steps(n, seed):
    """Quantiser steps that stress the reciprocal-and-correction quotient:
    mantissas of all ones and one unit from it, one unit above a power of two,
    small integers and halves, the ends of its range [2^-20, 2^20] and the
    floats just outside them (which take the division), then log-uniform
    steps over the range."""
    f = np.float32
    one_minus = np.nextafter(f(2), f(0))
    base = [f(2.0) ** k * m for k in (-20, -7, 0, 3, 5, 19) for m in
            (one_minus, np.nextafter(one_minus, f(0)), np.nextafter(f(1), f(2)), f(1.5))]
    base += [f(v) for v in (1, 3, 7, 28, 29.25, 63.5, 105.25, 0.1, 0.37, 13.25)]
    base += [f(2.0 ** -20), f(2.0 ** 20), np.nextafter(f(2.0 ** -20), f(0)), np.nextafter(f(2.0 ** 20), f(np.inf))]
    rng = np.random.default_rng(seed)
    rest = (2.0 ** rng.uniform(-20, 20, n - len(base))).astype(np.float32)
    return np.concatenate([np.array(base, np.float32), rest])


def test_quantiser_reciprocal_path_exact():
    """Steps in [2^-20, 2^20] quantise through the step's reciprocal and two
    FMA corrections of the quotient: on subbands large enough for the
    single-subband path, with values at and a few float32 steps around every
    (k + 1/2) step and random values, indices equal the oracle's FP32
    quantiser (correctly rounded division) for 256 such steps and for steps
    just outside the range."""
    H, W, J, dirs, B = 1024, 1024, 1, [4], 64
    table = geo.subband_table(H, W, J, dirs)
    steps = np.ones((B, len(table)), np.float32)
    steps[:, 1:] = _tricky_steps(B * (len(table) - 1), 11).reshape(B, len(table) - 1)
    rng = np.random.default_rng(12)
    n = table[-1].offset + table[-1].size
    c = np.empty((B, n), np.float32)
    for b in range(B):
        c[b] = _near_half_integers(table, steps[b], 1, 100 + b)[0]
        # a quarter of every subband: random bits with quotients up to 2^25
        for sb, st in zip(table[1:], steps[b, 1:]):
            m = sb.size // 4
            q = (2.0 ** rng.uniform(-3, 25, m)) * rng.choice([-1.0, 1.0], m)
            c[b, sb.offset:sb.offset + m] = (q * np.float64(st)).astype(np.float32)
    plan = _plan(H, W, J, dirs, B)
    idx, _ = plan.quantize(_dev(c), _dev(steps))
    idx_h = idx.cpu().numpy()
    for b in range(B):
        q_ref, _ = oq.quantize32(c[b], steps[b], table)
        np.testing.assert_array_equal(idx_h[b], q_ref)


def test_quantise_gpu_coefficients_mismatch_rate():
    """Indices from the GPU's own coefficients differ only at rounding boundaries."""
    H, W, J, dirs = 256, 256, 2, [8, 4]
    x = synth.luma_edges(H, W)[None].astype(np.float32)
    plan = _plan(H, W, J, dirs, 1)
    table = geo.subband_table(H, W, J, dirs)
    steps = np.full(len(table), 16.0, np.float32)
    idx, _ = plan.quantize(plan.forward(_dev(x)), _dev(steps))
    q_ref, _ = oq.quantize64(oct.forward(x[0].astype(np.float64), J, dirs), steps.astype(np.float64), table)
    q = idx.cpu().numpy()[0]
    assert np.mean(q != q_ref) < 1e-3
    assert np.abs(q.astype(int) - q_ref).max() <= 1


ACASES = [c for c in CASES if c[0] in ("c1", "ragged", "mixed", "deep6", "oddlow", "min8", "wide")]


@pytest.mark.parametrize("name,H,W,J,dirs,B", ACASES, ids=[c[0] for c in ACASES])
def test_adjoint_parity(name, H, W, J, dirs, B):
    _show(name, H=H, W=W, J=J, dirs=dirs, B=B)
    rng = np.random.default_rng(11)
    plan = _plan(H, W, J, dirs, B)
    g = rng.standard_normal((B, plan.ncoef)).astype(np.float32)
    y = rng.standard_normal((B, H, W)).astype(np.float32)
    fa = plan.forward_adjoint(_dev(g)).cpu().numpy()
    ia = plan.inverse_adjoint(_dev(y)).cpu().numpy()
    for b in range(B):
        want = oct.forward_adjoint(g[b].astype(np.float64), H, W, J, dirs)
        assert np.abs(fa[b] - want).max() <= TOL * max(1.0, np.abs(want).max())
        want = oct.inverse_adjoint(y[b].astype(np.float64), H, W, J, dirs)
        assert np.abs(ia[b] - want).max() <= TOL * max(1.0, np.abs(want).max())


def test_deterministic_repeat():
    H, W, J, dirs, B = 480, 640, 3, [16, 8, 4], 3
    x = _dev(_frames("c2", H, W, B))
    plan = _plan(H, W, J, dirs, B)
    a = plan.forward(x).clone()
    b = plan.forward(x).clone()
    assert torch.equal(a, b)
    assert torch.equal(plan.inverse(a), plan.inverse(b))


def test_empty_batch():
    plan = _plan(256, 256, 2, [8, 4], 0)
    out = plan.forward(torch.empty((0, 256, 256), device="cuda"))
    assert out.shape == (0, plan.ncoef)


def test_full_1080p_batch_sampled_planes():
    """The benchmark launch: 48 planes of 1080p (16 YCoCg frames), J=4, 32/16/8/8.

    The oracle runs whole planes; four planes of the batch are compared
    element by element, and the round trip is checked on every plane.
    """
    H, W, J, dirs, B = 1080, 1920, 4, [32, 16, 8, 8], 48
    _show("c3-full", H=H, W=W, J=J, dirs=dirs, B=B)
    x = clips.clip_planes(B // 3, H, W, 3)
    plan = _plan(H, W, J, dirs, B)
    xd = _dev(x)
    coef = plan.forward(xd)
    rec = plan.inverse(coef)
    rt = (rec - xd).abs().amax(dim=(1, 2)).cpu().numpy()
    assert rt.max() <= TOL, rt
    coef_h = coef.cpu().numpy()
    for b in (0, 1, 2, B - 1):
        ref = oct.forward(x[b].astype(np.float64), J, dirs)
        assert np.abs(coef_h[b] - ref).max() <= TOL, b
    # the benchmarked codec step: fused encoder and decoder with per-subband
    # steps; the indices are the oracle quantiser's on the GPU coefficients,
    # and the decoder output is the oracle's inverse of the oracle's
    # dequantisation of those indices
    table = geo.subband_table(H, W, J, dirs)
    steps = synth.subband_steps(plan.nsub, 3, 3)
    steps_b = np.stack([steps[b % 3] for b in range(B)]).astype(np.float32)
    idx, side = plan.encode(xd, _dev(steps_b))
    dec = plan.decode(idx, _dev(steps_b), side).cpu().numpy()
    idx_h, side_h = idx.cpu().numpy(), side.cpu().numpy()
    for b in (1, B - 1):
        q_ref, s_ref = oq.quantize32(coef_h[b], steps_b[b], table)
        np.testing.assert_array_equal(idx_h[b], q_ref)
        np.testing.assert_array_equal(side_h[b], s_ref)
        d_ref = oq.dequantize32(q_ref, steps_b[b], s_ref, table)
        rec_ref = oct.inverse(d_ref.astype(np.float64), H, W, J, dirs)
        assert np.abs(dec[b] - rec_ref).max() <= TOL, b
