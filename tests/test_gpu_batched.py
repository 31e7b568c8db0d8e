"""GPU tests of the batched form (one graph launch of grouped kernels).

Mixed streams of uneven resolution, LP depth and direction counts run
forward + quantise + dequantise + inverse in one launch; the result must be
bit-identical to the per-stream plain launches of the same plan, and agree
with the oracle.
"""
import json
import os
import time

import numpy as np
import pytest
import torch

from oracle import ct as oct
from oracle import geometry as geo
from oracle import quant as oq
from paper_1510_00561_amd import synth

pytestmark = pytest.mark.gpu

STREAMS = [
    (240, 320, 2, [8, 8], 3),
    (480, 640, 3, [16, 8, 8], 3),
    (720, 1280, 4, [16, 8, 8, 8], 1),
    (240, 320, 4, [8, 8, 8, 8], 3),
    (70, 90, 3, [16, 8, 4], 2),
    (64, 96, 2, [4, 32], 1),
    (256, 256, 2, [8, 4], 1),
    (40, 40, 3, [8, 4, 4], 3),      # odd coefficient count
    (4, 4, 1, [8], 2),              # smallest frame
    (128, 128, 1, [64], 1),         # six tree levels: three per pass, then one
]


def _streams(seed=0):
    from paper_1510_00561_amd import ct
    rng = np.random.default_rng(seed)
    out = []
    for H, W, J, dirs, B in STREAMS:
        planes = rng.uniform(0, 255, (B, H, W)).astype(np.float32)
        nsub = int(ct.layout(H, W, J, dirs)[0].nsub)
        steps = rng.integers(4, 65, size=(B, nsub)).astype(np.float32)
        out.append(dict(height=H, width=W, levels=J, dirs=dirs,
                        planes=torch.from_numpy(planes).cuda(), steps=torch.from_numpy(steps).cuda()))
    return out


def _snapshot(plan):
    return [{k: s[k].clone() for k in ("coeffs", "idx", "side", "deq", "out") if s[k] is not None}
            for s in plan.streams]


def _same(a, b):
    for x, y in zip(a, b):
        for k in x:
            assert torch.equal(x[k], y[k]), k


def test_batched_equals_plain_and_replays():
    from paper_1510_00561_amd import ct
    print("[batched] graph plan over", len(STREAMS), "streams", flush=True)
    plan = ct.Batched(_streams(), graph=True)
    info = plan.info()
    print("[batched] plan", info, flush=True)
    assert info["graph"] == 1 and info["streams"] == len(STREAMS)
    plan.run_plain()
    torch.cuda.synchronize()
    print("[batched] plain launches done", flush=True)
    plain = _snapshot(plan)
    for s in plan.streams:
        for k in ("coeffs", "idx", "side", "deq", "out"):
            s[k].zero_()
    for rep in range(3):
        t0 = time.perf_counter()
        plan.run()
        torch.cuda.synchronize()
        print(f"[batched] graph replay {rep}: {1e3 * (time.perf_counter() - t0):.2f} ms", flush=True)
        _same(plain, _snapshot(plan))
        # eager work between replays, then wipe the outputs
        torch.cuda.synchronize()
        for s in plan.streams:
            s["out"].fill_(-1.0)
    plan.close()


def test_batched_without_graph_matches():
    from paper_1510_00561_amd import ct
    plan = ct.Batched(_streams(1), graph=False)
    plan.run()
    torch.cuda.synchronize()
    a = _snapshot(plan)
    plan.run_plain()
    torch.cuda.synchronize()
    _same(a, _snapshot(plan))
    plan.close()


def test_batched_parity_with_oracle():
    from paper_1510_00561_amd import ct
    plan = ct.Batched(_streams(2), graph=True)
    plan.run()
    torch.cuda.synchronize()
    for (H, W, J, dirs, B), s in zip(STREAMS, plan.streams):
        # every stream, the 1280x720 depth-4 one (padded to 736 rows) included
        print(f"[batched] oracle check {H}x{W} J={J} dirs={dirs}", flush=True)
        table = geo.subband_table(H, W, J, dirs)
        x = s["planes"].cpu().numpy()
        coeffs = s["coeffs"].cpu().numpy()
        idx = s["idx"].cpu().numpy()
        deq = s["deq"].cpu().numpy()
        out = s["out"].cpu().numpy()
        steps = s["steps"].cpu().numpy()
        for b in range(min(B, 2)):
            ref = oct.forward(x[b].astype(np.float64), J, dirs)
            assert np.abs(coeffs[b] - ref).max() <= 1e-3
            q, side = oq.quantize32(coeffs[b], steps[b], table)
            np.testing.assert_array_equal(idx[b], q)
            np.testing.assert_array_equal(deq[b], oq.dequantize32(q, steps[b], side, table))
            rec = oct.inverse(deq[b].astype(np.float64), H, W, J, dirs)
            assert np.abs(out[b] - rec).max() <= 1e-3
    plan.close()


@pytest.fixture(autouse=True)
def _forget_tuning():
    """Tuned tile shapes live in a per-process table: start and leave every
    test of this file with the defaults."""
    from paper_1510_00561_amd import ct
    ct.autotune_clear()
    yield
    ct.autotune_clear()


def _tune_keys(streams):
    """(autotune cache key, l) of every LP level with three or more DFB tree
    levels in `streams` (the levels that run split passes), one entry per
    stream and level."""
    from paper_1510_00561_amd import ct
    arch = torch.cuda.get_device_properties(0).gcnArchName
    keys = []
    for H, W, J, dirs, B in streams:
        lay = ct.layout(H, W, J, dirs)[0]
        for j in range(1, J + 1):
            l = int(np.log2(dirs[j - 1]))
            if l >= 3:
                keys.append((f"{arch}|split_tune|{lay.pad_h >> (j - 1)}x{lay.pad_w >> (j - 1)}|l{l}|b{B}", l))
    return keys


def _valid_code(v):
    """Tree levels per pass in bits 0-3, block height mode in bits 4-5 (0
    default, 1 short, 2 tall, 3 explicit rows in bits 8-15, units of 4)."""
    grp, hm, rows = v & 15, (v >> 4) & 3, ((v >> 8) & 255) * 4
    if v >> 16 or v & 0xc0 or not 1 <= grp <= 3:
        return False
    return 32 <= rows <= 1020 if hm == 3 else rows == 0


def test_autotuned_plan(tmp_path, monkeypatch):
    from paper_1510_00561_amd import ct
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("CT_AUTOTUNE_CACHE", str(cache))
    plan = ct.Batched(_streams(3), graph=True, autotune=True)
    info = plan.info()
    assert info["autotuned"] == 1
    assert info["levels_paired"] + info["levels_single"] + info["levels_triple"] > 0
    assert cache.exists()
    entries = json.loads(cache.read_text())
    assert entries and all(_valid_code(v) for v in entries.values())
    assert {k for k, _ in _tune_keys(STREAMS)} <= set(entries)
    plan.run()
    torch.cuda.synchronize()
    tuned = _snapshot(plan)
    plan.close()
    ref = ct.Batched(_streams(3), graph=True)
    ref.run()
    torch.cuda.synchronize()
    _same(tuned, _snapshot(ref))
    ref.close()


def test_split_tile_shapes_are_bit_identical(tmp_path, monkeypatch):
    """Every tile-shape choice of the autotuner (tree levels per pass, row-block
    height) computes the same float32 operations in the same order, so the
    codec's output bits do not depend on the cache."""
    from paper_1510_00561_amd import ct
    keys = _tune_keys(STREAMS)
    deep = [l for _, l in keys if l >= 4]
    assert deep
    snaps = []
    # codes: tree levels per pass in bits 0-3, block height in bits 4-5
    # (0 default, 1 short, 2 tall, 3 explicit rows / 4 in bits 8-15)
    for code in (1, 2, 3, 1 | 16, 3 | 16, 2 | 32, 3 | 32, 3 | 48 | (192 // 4) << 8, 1 | 48 | (32 // 4) << 8,
                 2 | 48 | (248 // 4) << 8):
        cache = tmp_path / f"forced{code}.json"
        cache.write_text(json.dumps({k: code for k, _ in keys}))
        monkeypatch.setenv("CT_AUTOTUNE_CACHE", str(cache))
        plan = ct.Batched(_streams(5), graph=True, autotune=True)
        info = plan.info()
        grp, hm = code & 15, (code >> 4) & 3
        # a level with l tree levels runs at most l - 2 of them per pass
        want = {1: 0, 2: 0, 3: 0}
        for l in deep:
            want[min(grp, l - 2)] += 1
        assert (info["levels_single"], info["levels_paired"], info["levels_triple"]) == (want[1], want[2], want[3])
        assert info["levels_short_blocks"] == (len(keys) if hm == 1 else 0)
        assert info["levels_tall_blocks"] == (len(keys) if hm == 2 else 0)
        assert info["levels_sized_blocks"] == (len(keys) if hm == 3 else 0)
        plan.run()
        torch.cuda.synchronize()
        snaps.append(_snapshot(plan))
        plan.close()
        print(f"[batched] tune code {code} done", flush=True)
    for s in snaps[1:]:
        _same(snaps[0], s)


def test_fused_plan_equals_encode_decode():
    """A fused plan (grouped launches, one graph) gives each stream exactly
    what ct_encode and ct_decode give it alone, and its plain launches the
    same again."""
    from paper_1510_00561_amd import ct
    streams = _streams(4)
    plan = ct.Batched(streams, graph=True, fused=True)
    assert all(s["coeffs"] is None and s["deq"] is None for s in plan.streams)
    plan.run()
    torch.cuda.synchronize()
    graph = _snapshot(plan)
    plan.run_plain()
    torch.cuda.synchronize()
    _same(graph, _snapshot(plan))
    for (H, W, J, dirs, B), s, g in zip(STREAMS, plan.streams, graph):
        print(f"[batched] fused {H}x{W} J={J} dirs={dirs}", flush=True)
        single = ct.Plan(H, W, J, dirs, B, "cuda")
        idx, side = single.encode(s["planes"], s["steps"])
        out = single.decode(idx, s["steps"], side)
        torch.cuda.synchronize()
        assert torch.equal(g["idx"], idx) and torch.equal(g["side"], side)
        assert torch.equal(g["out"], out)
    plan.close()


def test_per_call_autotune_keeps_the_bits(tmp_path, monkeypatch):
    """ct_autotune records tile shapes that the per-call entry points then use:
    the transform and the fused codec give the same bits before and after, and
    a plan built afterwards without tuning takes the same choices."""
    from paper_1510_00561_amd import ct
    monkeypatch.setenv("CT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    ct.autotune_clear()
    H, W, J, dirs, B = 240, 320, 2, [32, 16], 3
    x = torch.from_numpy(np.random.default_rng(5).uniform(0, 255, (B, H, W)).astype(np.float32)).cuda()
    steps = torch.from_numpy(np.random.default_rng(6).integers(4, 65, ct.layout(H, W, J, dirs)[0].nsub)
                             .astype(np.float32)).cuda()
    plan = ct.Plan(H, W, J, dirs, B, "cuda")
    coef0 = plan.forward(x).clone()
    idx0, side0 = (t.clone() for t in plan.encode(x, steps))
    out0 = plan.decode(idx0, steps, side0).clone()
    plan.autotune()
    entries = json.loads((tmp_path / "tune.json").read_text())
    assert len(entries) == 2 and all(_valid_code(v) for v in entries.values())
    coef1 = plan.forward(x)
    idx1, side1 = plan.encode(x, steps)
    out1 = plan.decode(idx1, steps, side1)
    torch.cuda.synchronize()
    assert torch.equal(coef0, coef1) and torch.equal(idx0, idx1) and torch.equal(out0, out1)
    steps_b = steps.unsqueeze(0).expand(B, -1).contiguous()
    bt = ct.Batched([dict(height=H, width=W, levels=J, dirs=dirs, planes=x, steps=steps_b)], graph=True)
    info = bt.info()
    tuned = sum(1 for v in entries.values() if (v >> 4) & 3)
    assert info["levels_short_blocks"] + info["levels_tall_blocks"] + info["levels_sized_blocks"] == tuned
    bt.close()
