"""GPU parity of the variant filters and LP reconstruction against the oracle.

Variants (ct_geom.filters / .recon): the LeGall 5/3 pair for the LP and the
fan filters, and the Burt-Adelson LP reconstruction. The same tolerances as
the paper's transform: FP32 coefficients and reconstructions within max-abs
1e-3 of the FP64 oracle on the 0-255 scale (adjoints: relative 1e-5 of the
output's largest magnitude, as their values are not on the pixel scale).
"""
import numpy as np
import pytest
import torch

from oracle import ct as oct
from oracle import geometry as geo
from oracle import quant as oq

pytestmark = pytest.mark.gpu

TOL = 1e-3
VARIANTS = [("53", "dual"), ("53", "ba"), ("97", "ba")]
SHAPES = [
    ("ragged", 70, 90, 3, [16, 8, 4], 2),      # padded to 72 x 96
    ("split3", 96, 128, 2, [32, 8], 1),        # three tree levels in one pass at level 1
    ("dirs64", 64, 64, 1, [64], 1),            # two passes of three
]


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _plan(H, W, J, dirs, B, f, r):
    from paper_1510_00561_amd import ct
    return ct.Plan(H, W, J, dirs, B, "cuda", filters=f, recon=r)


def _x(H, W, B, seed):
    return np.random.default_rng(seed).uniform(0, 255, (B, H, W)).astype(np.float32)


@pytest.mark.parametrize("f,r", VARIANTS, ids=[f"{f}-{r}" for f, r in VARIANTS])
@pytest.mark.parametrize("name,H,W,J,dirs,B", SHAPES, ids=[s[0] for s in SHAPES])
def test_variant_forward_inverse(f, r, name, H, W, J, dirs, B):
    print(f"[variant] {name} filters={f} recon={r}", flush=True)
    x = _x(H, W, B, 41)
    plan = _plan(H, W, J, dirs, B, f, r)
    coef = plan.forward(_dev(x)).cpu().numpy()
    ref = np.stack([oct.forward(x[b].astype(np.float64), J, dirs, filters=f) for b in range(B)])
    assert np.abs(coef - ref).max() <= TOL
    # the inverse of perturbed oracle coefficients separates the two
    # reconstructions (on exact coefficients they agree)
    noisy = (ref + np.random.default_rng(42).uniform(-3, 3, ref.shape)).astype(np.float32)
    rec = plan.inverse(_dev(noisy)).cpu().numpy()
    for b in range(B):
        want = oct.inverse(noisy[b].astype(np.float64), H, W, J, dirs, filters=f, recon=r)
        assert np.abs(rec[b] - want).max() <= TOL
        other = oct.inverse(noisy[b].astype(np.float64), H, W, J, dirs, filters=f,
                            recon="dual" if r == "ba" else "ba")
        assert np.abs(rec[b] - other).max() > 10 * TOL


@pytest.mark.parametrize("f,r", VARIANTS, ids=[f"{f}-{r}" for f, r in VARIANTS])
def test_variant_codec_round_trip(f, r):
    """Fused encoder and decoder: indices bit-exact given the oracle's FP32
    quantiser on the GPU's own coefficients, and the decoded planes against
    the oracle's inverse of the dequantised indices."""
    H, W, J, dirs, B = 70, 90, 3, [16, 8, 4], 2
    x = _x(H, W, B, 43)
    table = geo.subband_table(H, W, J, dirs)
    steps = np.random.default_rng(44).integers(4, 33, len(table)).astype(np.float32)
    plan = _plan(H, W, J, dirs, B, f, r)
    coef = plan.forward(_dev(x))
    idx, side = plan.encode(_dev(x), _dev(steps))
    out = plan.decode(idx, _dev(steps), side).cpu().numpy()
    coef_h, idx_h, side_h = coef.cpu().numpy(), idx.cpu().numpy(), side.cpu().numpy()
    for b in range(B):
        q_ref, side_ref = oq.quantize32(coef_h[b], steps, table)
        np.testing.assert_array_equal(idx_h[b], q_ref)
        deq = oq.dequantize32(q_ref, steps, side_ref, table).astype(np.float64)
        want = oct.inverse(deq, H, W, J, dirs, filters=f, recon=r)
        assert np.abs(out[b] - want).max() <= TOL


@pytest.mark.parametrize("f,r", VARIANTS, ids=[f"{f}-{r}" for f, r in VARIANTS])
def test_variant_adjoints(f, r):
    H, W, J, dirs, B = 70, 90, 3, [16, 8, 4], 1
    rng = np.random.default_rng(45)
    n = geo.ncoef(H, W, J, dirs)
    g = rng.standard_normal((B, n)).astype(np.float32)
    y = rng.standard_normal((B, H, W)).astype(np.float32)
    plan = _plan(H, W, J, dirs, B, f, r)
    fa = plan.forward_adjoint(_dev(g)).cpu().numpy()[0]
    ia = plan.inverse_adjoint(_dev(y)).cpu().numpy()[0]
    want_fa = oct.forward_adjoint(g[0].astype(np.float64), H, W, J, dirs, filters=f)
    want_ia = oct.inverse_adjoint(y[0].astype(np.float64), H, W, J, dirs, filters=f, recon=r)
    assert np.abs(fa - want_fa).max() <= 1e-5 * np.abs(want_fa).max()
    assert np.abs(ia - want_ia).max() <= 1e-5 * np.abs(want_ia).max()


def test_variants_in_one_batched_graph():
    """Streams of every variant in one plan: bit-identical to their plain
    per-stage runs, and each against the oracle."""
    from paper_1510_00561_amd import ct
    H, W, J, dirs = 70, 90, 3, [16, 8, 4]
    table = geo.subband_table(H, W, J, dirs)
    steps = np.random.default_rng(46).integers(4, 33, len(table)).astype(np.float32)
    streams = []
    kinds = [("97", "dual")] + VARIANTS
    for i, (f, r) in enumerate(kinds):
        streams.append(dict(height=H, width=W, levels=J, dirs=dirs, planes=_dev(_x(H, W, 1, 50 + i)),
                            steps=_dev(steps), filters=f, recon=r))
    bt = ct.Batched(streams, graph=True, fused=True)
    bt.run()
    got = [(s["idx"].clone(), s["out"].clone()) for s in bt.streams]
    bt.run_plain()
    torch.cuda.synchronize()
    for (gi, go), s, (f, r) in zip(got, bt.streams, kinds):
        assert torch.equal(gi, s["idx"]) and torch.equal(go, s["out"])
        x = s["planes"].cpu().numpy()[0].astype(np.float64)
        coef = oct.forward(x, J, dirs, filters=f)
        q_ref, side_ref = oq.quantize32(coef.astype(np.float32), steps, table)
        mism = np.mean(gi.cpu().numpy()[0] != q_ref)
        assert mism < 1e-3, (f, r, mism)
        deq = oq.dequantize32(gi.cpu().numpy()[0], steps, s["side"].cpu().numpy()[0], table)
        want = oct.inverse(deq.astype(np.float64), H, W, J, dirs, filters=f, recon=r)
        assert np.abs(go.cpu().numpy()[0] - want).max() <= TOL
