"""GPU tests of the fused encoder and decoder (ct_encode, ct_decode).

ct_encode must give the indices and side info of ct_forward + ct_quantize,
and ct_decode the planes of ct_dequantize + ct_inverse, bit for bit: they run
the same float32 operations on the same values, only without the float
coefficients in HBM. Against the FP64 oracle the fused round trip meets the
same bounds as the separate calls (indices differ from the oracle's only at
rounding boundaries; reconstructions within 1e-3).
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import ct as oct
from oracle import geometry as geo
from oracle import quant as oq
from tests import clips

pytestmark = pytest.mark.gpu

CASES = [
    ("c1", 256, 256, 2, [8, 4], 1),
    ("tiny", 16, 16, 2, [8, 4], 2),
    ("ragged", 70, 90, 3, [16, 8, 4], 2),
    ("c2", 480, 640, 3, [16, 8, 4], 3),
    ("dirs64", 128, 128, 1, [64], 1),
    ("mixed", 64, 96, 2, [4, 32], 2),
    ("deep6", 192, 256, 6, [8, 8, 4, 4, 4, 4], 1),
    ("c3", 1080, 1920, 4, [32, 16, 8, 8], 3),
    ("oddlow", 40, 40, 3, [8, 4, 4], 3),
    ("min8", 4, 4, 1, [8], 2),
    ("wide", 24, 200, 2, [16, 4], 2),
]


def _frames(name, H, W, B):
    if name in ("c2", "c3"):
        return clips.clip_planes(max(1, B // 3), H, W, {"c2": 2, "c3": 3}[name])[:B]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    return rng.uniform(0, 255, (B, H, W)).astype(np.float32)


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


@pytest.mark.parametrize("name,H,W,J,dirs,B", CASES, ids=[c[0] for c in CASES])
def test_fused_equals_separate_calls(name, H, W, J, dirs, B):
    from paper_1510_00561_amd import ct
    print(f"[fused] {name} {H}x{W} J={J} dirs={dirs} B={B}", flush=True)
    plan = ct.Plan(H, W, J, dirs, B, "cuda")
    x = _dev(_frames(name, H, W, B))
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 1)
    steps = _dev(rng.integers(1, 65, size=(B, plan.nsub)).astype(np.float32))
    # separate calls
    coef = plan.forward(x)
    idx_ref, side_ref = plan.quantize(coef, steps)
    rec_ref = plan.inverse(plan.dequantize(idx_ref, steps, side_ref))
    # fused encoder, without and with the float coefficients
    idx, side = plan.encode(x, steps)
    assert torch.equal(idx, idx_ref) and torch.equal(side, side_ref)
    coef2 = torch.full_like(coef, float("nan"))
    idx2, side2 = plan.encode(x, steps, coeffs=coef2)
    assert torch.equal(idx2, idx_ref) and torch.equal(side2, side_ref)
    assert torch.equal(coef2, coef)
    # fused decoder
    rec = plan.decode(idx_ref, steps, side_ref)
    assert torch.equal(rec, rec_ref)
    # one shared step row
    idx3, side3 = plan.encode(x, steps[0])
    idx3_ref, _ = plan.quantize(coef, steps[0])
    assert torch.equal(idx3, idx3_ref)
    assert torch.equal(plan.decode(idx3, steps[0], side3),
                       plan.inverse(plan.dequantize(idx3_ref, steps[0], side3)))
    torch.cuda.synchronize()


def test_fused_round_trip_against_oracle():
    from paper_1510_00561_amd import ct
    H, W, J, dirs, B = 480, 640, 3, [16, 8, 4], 2
    x = _frames("c2", H, W, B)
    plan = ct.Plan(H, W, J, dirs, B, "cuda")
    table = geo.subband_table(H, W, J, dirs)
    steps = np.full((B, plan.nsub), 8.0, np.float32)
    idx, side = plan.encode(_dev(x), _dev(steps))
    rec = plan.decode(idx, _dev(steps), side).cpu().numpy()
    idx = idx.cpu().numpy()
    for b in range(B):
        c = oct.forward(x[b].astype(np.float64), J, dirs)
        q, s = oq.quantize64(c, steps[b].astype(np.float64), table)
        assert np.mean(idx[b] != q) < 1e-3
        assert np.abs(idx[b].astype(int) - q).max() <= 1
        # the oracle decodes the GPU's own indices and side info
        d = oq.dequantize64(idx[b].astype(np.int64), steps[b].astype(np.float64),
                            side[b].cpu().numpy().astype(np.float64), table)
        ref = oct.inverse(d, H, W, J, dirs)
        assert np.abs(rec[b] - ref).max() <= 1e-3


@pytest.mark.parametrize("serial", ["0", "1"])
def test_encode_decode_captured_in_a_graph(serial, monkeypatch):
    """ct_encode + ct_decode captured into one HIP graph (the level-1 split
    passes fork onto the library's second stream and join back inside the
    capture), replayed three times with eager work in between: every replay
    equals the eager results bit for bit, with and without the fork."""
    from paper_1510_00561_amd import ct
    monkeypatch.setenv("CT_SERIAL_LEVELS", serial)
    H, W, J, dirs, B = 240, 320, 3, [32, 16, 8], 3
    print(f"[fused] graph capture serial={serial}", flush=True)
    rng = np.random.default_rng(77)
    x = torch.from_numpy(rng.uniform(0, 255, (B, H, W)).astype(np.float32)).cuda()
    plan = ct.Plan(H, W, J, dirs, B, "cuda")
    steps = torch.from_numpy(rng.integers(4, 65, plan.nsub).astype(np.float32)).cuda()
    idx = torch.empty((B, plan.ncoef), dtype=torch.int16, device="cuda")
    side = torch.empty((B, 2), dtype=torch.float32, device="cuda")
    out = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    plan.encode(x, steps, idx, side)
    plan.decode(idx, steps, side, out=out)
    torch.cuda.synchronize()
    ref = (idx.clone(), side.clone(), out.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            plan.encode(x, steps, idx, side)
            plan.decode(idx, steps, side, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.encode(x, steps, idx, side)
        plan.decode(idx, steps, side, out=out)
    for _ in range(3):
        idx.zero_()
        side.zero_()
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(idx, ref[0]) and torch.equal(side, ref[1]) and torch.equal(out, ref[2])
    del g
