"""ct_quantize_noalloc (static scratch, no workspace) against ct_quantize.

Two calls in a row on one device, the second on a smaller batch and another
geometry, each compared bit for bit with ct_quantize on the same input; the
second call reuses the scratch the first one left behind.
"""
import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import quant as oq
from paper_1510_00561_amd import ct, synth


def _case(H, W, J, dirs, B, seed):
    plan = ct.Plan(H, W, J, dirs, B, "cuda:0")
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(np.stack([synth.luma_edges(H, W, seed + b) for b in range(B)]).astype(np.float32)).cuda()
    coef = plan.forward(x)
    steps = torch.from_numpy(rng.integers(4, 65, size=(B, plan.nsub)).astype(np.float32)).cuda()
    return plan, coef, steps


@pytest.mark.gpu
def test_quantize_noalloc_matches_workspace_call():
    print("[no-alloc] case 1: 6 x 256x256 J=2 8/4", flush=True)
    cases = [(256, 256, 2, [8, 4], 6, 11), (70, 90, 3, [16, 8, 4], 2, 12)]
    for H, W, J, dirs, B, seed in cases:
        plan, coef, steps = _case(H, W, J, dirs, B, seed)
        idx_ref, side_ref = plan.quantize(coef, steps)
        idx, side = plan.quantize_noalloc(coef, steps)
        torch.cuda.synchronize()
        assert torch.equal(idx, idx_ref), f"indices differ at {H}x{W} batch {B}"
        assert torch.equal(side, side_ref), f"side info differs at {H}x{W} batch {B}"
        # and both equal the oracle's FP32 quantiser on the same coefficients
        table = geo.subband_table(H, W, J, dirs)
        c = coef.cpu().numpy()
        s = steps.cpu().numpy()
        for b in range(B):
            q_ref, sd = oq.quantize32(c[b], s[b], table)
            assert np.array_equal(idx[b].cpu().numpy(), q_ref)
            assert np.array_equal(side[b].cpu().numpy(), sd)
        print(f"[no-alloc] {H}x{W} J={J} batch {B}: identical", flush=True)


@pytest.mark.gpu
def test_quantize_noalloc_shared_row_and_limit():
    plan, coef, steps = _case(64, 96, 2, [4, 32], 3, 21)
    row = steps[0].contiguous()
    idx_ref, side_ref = plan.quantize(coef, row)
    idx, side = plan.quantize_noalloc(coef, row)
    torch.cuda.synchronize()
    assert torch.equal(idx, idx_ref) and torch.equal(side, side_ref)
    big = ct.Plan(16, 16, 1, [4], 1025, "cuda:0")
    c = torch.zeros((1025, big.ncoef), dtype=torch.float32, device="cuda:0")
    s = torch.ones(big.nsub, dtype=torch.float32, device="cuda:0")
    with pytest.raises(ct.CTError) as e:
        big.quantize_noalloc(c, s)
    assert e.value.code == -3
