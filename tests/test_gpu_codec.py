"""GPU tests of the codec stages after the quantiser: contourlet-domain motion
compensation of P-frames (paper section 3.7) and the zero-run coder (section
3.8), bit-exact against the oracle on inputs generated on the host, and the
whole back end (vectors, P-frame components, symbols, DEFLATE) restoring the
indices exactly."""
import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import mc
from oracle import rle
from paper_1510_00561_amd import synth
from tests import clips

pytestmark = pytest.mark.gpu


def _plan(H, W, J, dirs, B):
    from paper_1510_00561_amd import ct
    return ct.Plan(H, W, J, dirs, B, "cuda")


def _idx(table, B, seed, density=1.0, lo=-32768, hi=32767):
    rng = np.random.default_rng(seed)
    n = table[-1].offset + table[-1].size
    v = rng.integers(lo, hi + 1, size=(B, n))
    return np.where(rng.random((B, n)) < density, v, 0).astype(np.int16)


MC_CASES = [
    (64, 96, 2, [8, 4], 2, 1, 1, 16),
    (70, 90, 3, [16, 8, 4], 2, 3, 1, 32767),  # vectors far beyond a component's size, factor 3
    (70, 90, 3, [16, 8, 4], 3, 1, 3, 16),   # padded; three planes share one vector field
    (64, 96, 2, [4, 32], 2, 2, 1, 16),      # chroma factor 2
    (40, 40, 3, [8, 4, 4], 3, 4, 1, 16),    # odd coefficient count, factor 4
    (128, 128, 1, [64], 1, 1, 1, 16),
    (240, 320, 4, [8, 8, 8, 8], 3, 1, 3, 16),
]


@pytest.mark.parametrize("H,W,J,dirs,B,n,group,vmax", MC_CASES)
def test_mc_residual_bit_exact(H, W, J, dirs, B, n, group, vmax):
    print(f"[codec] mc {H}x{W} J={J} dirs={dirs} B={B} n={n} group={group} |v| <= {vmax}", flush=True)
    table = geo.subband_table(H, W, J, dirs)
    plan = _plan(H, W, J, dirs, B)
    cur, prev = _idx(table, B, 1), _idx(table, B, 2)
    nby, nbx = -(-H * n // 16), -(-W * n // 16)
    rng = np.random.default_rng(3)
    mv = rng.integers(-vmax, vmax + 1, size=(-(-B // group), nby, nbx, 2)).astype(np.int16)
    cd, pd, md = (torch.from_numpy(a).cuda() for a in (cur, prev, mv))
    res = plan.mc_residual(cd, pd, md, n=n, group=group).cpu().numpy()
    for b in range(B):
        want = mc.residual_plane(cur[b], prev[b], table, J, mv[b // group], n)
        np.testing.assert_array_equal(res[b], want)
    # the decoder restores the indices, also in place
    rd = torch.from_numpy(res).cuda()
    back = plan.mc_residual(rd, pd, md, n=n, group=group, inverse=True)
    assert torch.equal(back, cd)
    plan.mc_residual(rd, pd, md, n=n, group=group, inverse=True, out=rd)
    assert torch.equal(rd, cd)


RLE_CASES = [
    (16, 16, 1, [4], 2),
    (64, 96, 2, [4, 32], 2),
    (70, 90, 3, [16, 8, 4], 3),
    (40, 40, 3, [8, 4, 4], 3),
    (4, 4, 1, [8], 2),
    (480, 640, 3, [16, 8, 4], 1),
]


@pytest.mark.parametrize("H,W,J,dirs,B", RLE_CASES)
@pytest.mark.parametrize("p_frame", [0, 1])
def test_rle_bit_exact(H, W, J, dirs, B, p_frame):
    print(f"[codec] rle {H}x{W} J={J} dirs={dirs} B={B} p={p_frame}", flush=True)
    table = geo.subband_table(H, W, J, dirs)
    plan = _plan(H, W, J, dirs, B)
    for density in (0.0, 0.02, 0.3, 1.0):
        idx = _idx(table, B, 10 + int(100 * density), density, -50, 50)
        sym, off = plan.rle_encode(torch.from_numpy(idx).cuda(), p_frame)
        sym, off = sym.cpu().numpy(), off.cpu().numpy()
        for b in range(B):
            want_sym, want_off = rle.encode_plane(idx[b], table, p_frame)
            np.testing.assert_array_equal(off[b], want_off)
            np.testing.assert_array_equal(sym[b, :off[b, -1]], want_sym)
            np.testing.assert_array_equal(plan.rle_decode_host(sym[b, :off[b, -1]], off[b], p_frame), idx[b])


def test_codec_back_end_on_clip_frames():
    """K-frame then P-frame of the synthetic clip at 640x480 (3 channels,
    chroma factor 1): fused encoder, motion search on Y, P-frame components,
    zero-run symbols and DEFLATE; decoding the bytes restores the indices."""
    from paper_1510_00561_amd import ct
    H, W, J, dirs = 480, 640, 3, [16, 8, 4]
    x = clips.clip_planes(2, H, W, 2)                      # [6, H, W]: two YCoCg frames
    plan = _plan(H, W, J, dirs, 3)
    steps = torch.full((plan.nsub,), 8.0, device="cuda")
    idx0, side0 = plan.encode(torch.from_numpy(x[:3]).cuda(), steps)
    idx1, side1 = plan.encode(torch.from_numpy(x[3:]).cuda(), steps)
    mv, _ = ct.motion_search(torch.from_numpy(x[3:4]).cuda(), torch.from_numpy(x[0:1]).cuda(), 8)
    res = plan.mc_residual(idx1, idx0, mv, n=1, group=3)
    table = geo.subband_table(H, W, J, dirs)
    for frame, p_frame in ((idx0, 0), (res, 1)):
        sym, off = plan.rle_encode(frame, p_frame)
        sym, off = sym.cpu().numpy(), off.cpu().numpy()
        host = frame.cpu().numpy()
        for b in range(3):
            s = sym[b, :off[b, -1]]
            ws, wo = rle.encode_plane(host[b], table, p_frame)
            np.testing.assert_array_equal(s, ws)
            blob, parts = ct.deflate_host(s, off[b], 0)
            back = ct.inflate_host(blob, parts, off[b], 0)
            np.testing.assert_array_equal(plan.rle_decode_host(back, off[b], p_frame), host[b])
    # the decoder side of the P-frame: prediction from frame 0's indices
    assert torch.equal(plan.mc_residual(res, idx0, mv, n=1, group=3, inverse=True), idx1)
    # the same vectors through the oracle
    want = mc.residual_plane(idx1[0].cpu().numpy(), idx0[0].cpu().numpy(), table, J, mv[0].cpu().numpy().astype(np.int64))
    np.testing.assert_array_equal(res[0].cpu().numpy(), want)
