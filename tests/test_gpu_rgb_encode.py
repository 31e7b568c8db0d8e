"""GPU parity of the fused RGB encoder (ct_encode_rgb).

ct_encode_rgb converts 8-bit RGB to Y, Co + 127, Cg + 127 (equations (1)-(3),
chroma kept at every sample) where the first LP level loads its rows, then
runs the fused encoder. Every colour value is a quarter integer below 2^10,
exact in float32, so the planes it filters are the very floats
ct_rgb_to_ycocg writes and the indices and side data must equal those of
ct_rgb_to_ycocg + ct_encode bit for bit. Against the oracle (FP64 colour
transform and CT, FP32 quantiser on the rounded coefficients), an index may
differ by one where a float32 coefficient sits within rounding of a
quantiser boundary: at most 1e-3 of them.
"""
import numpy as np
import pytest
import torch

from oracle import color
from oracle import ct as oct
from oracle import geometry as geo
from oracle import quant as oq
from paper_1510_00561_amd import ct

pytestmark = pytest.mark.gpu

# (name, frames, height, width, levels, dirs, filters)
CASES = [
    ("ragged", 2, 70, 90, 3, [16, 8, 4], "97"),     # padded to 72 x 96: mirrored rows and columns
    ("odd", 1, 45, 61, 2, [8, 4], "97"),            # odd sizes, padded to 48 x 64
    ("split3", 1, 96, 128, 2, [32, 8], "97"),       # three tree levels in one pass at level 1
    ("legall", 2, 70, 90, 3, [16, 8, 4], "53"),     # the 5/3 variant (other level-1 kernel taps)
    ("quant1", 2, 66, 100, 1, [4], "97"),           # four directions at level 1: indices stored by the RGB stage
]


def _rgb(F, H, W, seed):
    return np.random.default_rng(seed).integers(0, 256, size=(F, H, W, 3)).astype(np.uint8)


def _steps(H, W, J, dirs, seed):
    n = len(geo.subband_table(H, W, J, dirs))
    return np.random.default_rng(seed).integers(4, 33, n).astype(np.float32)


def _separate(plan, rgb_d, steps_d):
    """ct_rgb_to_ycocg (n = 1) + ct_encode on the planes stacked frame by frame."""
    y, co, cg = ct.rgb_to_ycocg(rgb_d, 1)
    planes = torch.stack([y, co, cg], 1).reshape(-1, plan.height, plan.width).contiguous()
    return plan.encode(planes, steps_d), planes


@pytest.mark.parametrize("name,F,H,W,J,dirs,f", CASES, ids=[c[0] for c in CASES])
def test_encode_rgb_equals_colour_then_encode(name, F, H, W, J, dirs, f):
    print(f"[rgb-encode] {name} F={F} {H}x{W} J={J} dirs={dirs} filters={f}", flush=True)
    rgb = _rgb(F, H, W, 60 + len(name))
    steps = _steps(H, W, J, dirs, 61)
    plan = ct.Plan(H, W, J, dirs, 3 * F, "cuda", filters=f)
    rgb_d = torch.from_numpy(rgb).cuda()
    steps_d = torch.from_numpy(steps).cuda()
    idx, side = plan.encode_rgb(rgb_d, steps_d)
    (idx_ref, side_ref), _ = _separate(plan, rgb_d, steps_d)
    assert torch.equal(idx, idx_ref)
    assert torch.equal(side, side_ref)
    # against the oracle
    table = geo.subband_table(H, W, J, dirs)
    idx_h, side_h = idx.cpu().numpy(), side.cpu().numpy()
    for fr in range(F):
        for k, plane in enumerate(color.encode_frame(rgb[fr], 1)):
            b = 3 * fr + k
            coef = oct.forward(plane.astype(np.float64), J, dirs, filters=f).astype(np.float32)
            q, s = oq.quantize32(coef, steps, table)
            d = np.abs(idx_h[b].astype(np.int32) - q)
            assert d.max() <= 1 and np.mean(d != 0) <= 1e-3, (b, d.max(), np.mean(d != 0))
            np.testing.assert_allclose(side_h[b], s, atol=1e-3)


def test_encode_rgb_per_plane_steps_and_reuse():
    """Per-plane steps (one row per plane, plane 3 f + k = channel k of frame
    f), two calls in a row on one plan, and a decode of the result."""
    F, H, W, J, dirs = 3, 64, 96, 2, [8, 4]
    n = len(geo.subband_table(H, W, J, dirs))
    plan = ct.Plan(H, W, J, dirs, 3 * F, "cuda")
    steps = np.random.default_rng(62).integers(4, 33, (3 * F, n)).astype(np.float32)
    steps_d = torch.from_numpy(steps).cuda()
    for seed in (63, 64):
        rgb_d = torch.from_numpy(_rgb(F, H, W, seed)).cuda()
        idx, side = plan.encode_rgb(rgb_d, steps_d)
        (idx_ref, side_ref), planes = _separate(plan, rgb_d, steps_d)
        assert torch.equal(idx, idx_ref) and torch.equal(side, side_ref)
        rec = plan.decode(idx, steps_d, side)
        # a coarse check that the indices carry the frames: decoded planes
        # within the quantiser's reach of the originals
        assert (rec - planes).abs().mean().item() < 8.0


def test_encode_rgb_full_hd():
    """The full-size workload: 16 frames of 1080 x 1920 (48 planes), 4 LP
    levels with 32/16/8/8 directions, as one call."""
    F, H, W, J, dirs = 16, 1080, 1920, 4, [32, 16, 8, 8]
    print(f"[rgb-encode] full HD F={F}", flush=True)
    plan = ct.Plan(H, W, J, dirs, 3 * F, "cuda")
    steps_d = torch.from_numpy(_steps(H, W, J, dirs, 65)).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(66)
    rgb_d = torch.randint(0, 256, (F, H, W, 3), dtype=torch.uint8, device="cuda", generator=g)
    idx, side = plan.encode_rgb(rgb_d, steps_d)
    (idx_ref, side_ref), _ = _separate(plan, rgb_d, steps_d)
    assert torch.equal(idx, idx_ref)
    assert torch.equal(side, side_ref)


def test_encode_rgb_rejects_a_batch_not_of_frames():
    plan = ct.Plan(64, 64, 2, [8, 4], 4, "cuda")
    with pytest.raises(ValueError):
        plan.encode_rgb(torch.zeros((1, 64, 64, 3), dtype=torch.uint8, device="cuda"),
                        torch.ones(plan.nsub, device="cuda"))


def test_encode_rgb_captured_in_a_graph():
    """ct_encode_rgb + ct_decode captured into one HIP graph (with the fork of
    the level-1 split passes), replayed three times with eager work in
    between: every replay equals the eager results bit for bit."""
    F, H, W, J, dirs = 2, 240, 320, 3, [32, 16, 8]
    print("[rgb-encode] graph capture", flush=True)
    plan = ct.Plan(H, W, J, dirs, 3 * F, "cuda")
    rgb_d = torch.from_numpy(_rgb(F, H, W, 67)).cuda()
    steps_d = torch.from_numpy(_steps(H, W, J, dirs, 68)).cuda()
    idx = torch.empty((3 * F, plan.ncoef), dtype=torch.int16, device="cuda")
    side = torch.empty((3 * F, 2), dtype=torch.float32, device="cuda")
    out = torch.empty((3 * F, H, W), dtype=torch.float32, device="cuda")
    plan.encode_rgb(rgb_d, steps_d, idx, side)
    plan.decode(idx, steps_d, side, out=out)
    torch.cuda.synchronize()
    ref = (idx.clone(), side.clone(), out.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            plan.encode_rgb(rgb_d, steps_d, idx, side)
            plan.decode(idx, steps_d, side, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.encode_rgb(rgb_d, steps_d, idx, side)
        plan.decode(idx, steps_d, side, out=out)
    for _ in range(3):
        idx.zero_()
        side.zero_()
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(idx, ref[0]) and torch.equal(side, ref[1]) and torch.equal(out, ref[2])
    del g
