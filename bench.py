"""Benchmark: contourlet forward + quantise + dequantise + inverse on 1080p frames.

One step is the whole hot path on one batch: 16 synthetic 1920x1080 RGB
frames, converted to YCoCg by the library beforehand (48 float32 planes: Y,
Co + 127, Cg + 127, padded to 1088 x 1920), LP 4 levels,
DFB 32/16/8/8 directions, per-subband quantisation steps drawn per channel
from 4..64. Inputs are resident in HBM before timing starts.

Prints one JSON line. `value` is frames/s (real 1080p frames). The line also
carries the effective HBM bandwidth of the step (algorithmic bytes / time),
the roofline of the dominant kernel from live per-launch HIP events, the
colour front end / back end and K-frame lowpass filter measured on the same
frames (outside the step), and the FP64 oracle timed on the host cores on a
bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "1080p frames/s for CT forward+inverse+quant; HBM GB/s as % of peak; batched vs plain"

H, W, J, DIRS = 1080, 1920, 4, [32, 16, 8, 8]
FRAMES = 16
PLANES = 3 * FRAMES

# kernel -> sources whose text defines it (a change invalidates its counters)
KERNEL_SOURCES = {   # the kernel's code and the host code that sets its launch shape (block heights)
    "lp_dfb12_analysis": ("ct_level.hip", "ct_stream_level.h", "ct_stream.h", "ct_kernels.h", "ct_api.cpp"),
    "dfb12_lp_synthesis": ("ct_level.hip", "ct_stream_level.h", "ct_stream.h", "ct_kernels.h", "ct_api.cpp"),
    "dfb_split_analysis": ("ct_level.hip", "ct_stream.h", "ct_stages.h", "ct_kernels.h", "ct_api.cpp"),
    "dfb_split_synthesis": ("ct_level.hip", "ct_stream.h", "ct_stages.h", "ct_kernels.h", "ct_api.cpp"),
    "dfb_split2_analysis": ("ct_level.hip", "ct_stream.h", "ct_stages.h", "ct_kernels.h", "ct_api.cpp"),
    "dfb_split2_synthesis": ("ct_level.hip", "ct_stream.h", "ct_stages.h", "ct_kernels.h", "ct_api.cpp"),
    "pad_fold": ("ct_level.hip",),
    "lowpass_partial": ("ct_quant.hip", "ct_quant_stages.h"),
    "quantize": ("ct_quant.hip", "ct_quant_stages.h"),
    "dequantize": ("ct_quant.hip", "ct_quant_stages.h"),
    "rgb_to_ycocg": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "ycocg_to_rgb": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "lowpass_diff": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "lowpass_undiff": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "motion_search": ("ct_motion.hip", "ct_motion.h", "ct_motion_api.cpp"),
}


def algorithmic_bytes_per_plane(ncoef):
    """Forward 4HW + 4n, quantise 4n + 2n, dequantise 2n + 4n, inverse 4n + 4HW."""
    return 8 * H * W + 20 * ncoef


def source_digest(name):
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES.get(name, ()):
        with open(os.path.join(ROOT, "paper_1510_00561_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(name, bytes_per_launch, summary="traffic_1080p.json"):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if current."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get("kernels", {}).get(name)
    if not ent or ent.get("source_sha256_16") != source_digest(name):
        return None
    return ent.get("hbm_bytes_per_launch")


def cpu_baseline(rgb_frame, steps_np, seconds_budget=30.0):
    """The FP64 oracle on one 1080p YCoCg frame (3 planes), single process."""
    import numpy as np
    from oracle import color
    from oracle import ct as oct
    from oracle import geometry as geo
    from oracle import quant as oq
    table = geo.subband_table(H, W, J, DIRS)
    planes_np = np.stack(color.encode_frame(rgb_frame, 1))
    t0 = time.perf_counter()
    n = 0
    for b in range(3):
        x = planes_np[b].astype(np.float64)
        c = oct.forward(x, J, DIRS)
        q, side = oq.quantize64(c, steps_np[b % 3].astype(np.float64), table)
        d = oq.dequantize64(q, steps_np[b % 3].astype(np.float64), side, table)
        oct.inverse(d, H, W, J, DIRS)
        n += 1
        if time.perf_counter() - t0 > seconds_budget:
            break
    dt = time.perf_counter() - t0
    frames = n / 3.0
    return {"value": frames / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} of the 3 planes of one 1080p YCoCg frame, forward+quantise+dequantise+inverse "
                      f"in FP64 NumPy, one process ({dt:.1f} s)"}


def ycocg_planes(rgb):
    """[B, H, W, 3] uint8 device frames -> [3B, H, W] float32 planes Y, Co + 127,
    Cg + 127 of each frame in turn (the library's colour stage, chroma factor 1)."""
    import torch
    from paper_1510_00561_amd import ct
    y, co, cg = ct.rgb_to_ycocg(rgb, 1)
    B, Hh, Ww = y.shape
    return torch.stack([y, co, cg], dim=1).reshape(3 * B, Hh, Ww).contiguous()


def front_back_stages(rgb, plan, idx, steps, n=4, check_factor1=True):
    """Colour front end and back end on the bench's frames (chroma factor n),
    and the K-frame lowpass filter and its inverse on the step's indices:
    per-kernel time from HIP events, achieved against HBM peak."""
    import torch
    from paper_1510_00561_amd import ct
    # Three buffer sets (2.6 GB) in rotation, and each kernel timed in a loop
    # of its own: a launch never finds its inputs in the 256 MB last-level
    # cache from an earlier launch, so the times are HBM times.
    sets = []
    for _ in range(3):
        r = rgb.clone()
        y, co, cg = ct.rgb_to_ycocg(r, n)
        sets.append((r, y, co, cg, ct.ycocg_to_rgb(y, co, cg, n)))
    work = idx.clone()
    torch.cuda.synchronize()
    ct.profile_enable(True, 8192)
    for i in range(3 * steps):
        r, y, co, cg, _ = sets[i % 3]
        ct.rgb_to_ycocg(r, n, y, co, cg)
    for i in range(3 * steps):
        _, y, co, cg, out = sets[i % 3]
        ct.ycocg_to_rgb(y, co, cg, n, out)
    for _ in range(steps):
        plan.lowpass_diff(work)
        plan.lowpass_diff(work, inverse=True)
    torch.cuda.synchronize()
    stats = ct.profile_collect()
    ct.profile_enable(False)
    del sets
    restored = bool(torch.equal(work, idx))
    exact = None
    if check_factor1:
        y1, co1, cg1 = ct.rgb_to_ycocg(rgb, 1)
        exact = bool(torch.equal(ct.ycocg_to_rgb(y1, co1, cg1, 1), rgb.float()))
    kern = {}
    for name, (cnt, tms, by) in stats.items():
        gbps = by / (tms / 1e3) / 1e9
        kern[name] = {"avg_launch_us": round(tms / cnt * 1e3, 2), "bytes_per_launch": by / cnt,
                      "achieved_gbps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
                      "traffic": measured_traffic("lowpass_diff" if name == "lowpass_undiff" else name,
                                                  by / cnt, "traffic_colour_1080p.json")}
    B, Hh, Ww, _ = rgb.shape
    return {"workload": f"{B} x {Ww}x{Hh} RGB frames, chroma factor {n}; K-frame lowpass filter and its "
                        f"inverse on the step's {idx.shape[0]} planes of indices",
            "bound": "hbm", "peak_gbps": HBM_PEAK_GBPS, "kernels": kern,
            "lowpass_roundtrip_exact": restored, "colour_roundtrip_exact_factor1": exact}


VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: 32-bit VALU lane-ops/s


def motion_stage(planes, steps, w=8):
    """Full-search block matching (16 x 16 blocks, +-w) of each Y plane of the
    batch against the one before: per-launch time from HIP events, against the
    VALU issue rate at one lane-op per candidate pixel (a packed 16-bit
    subtraction and a 16-bit dot product handle two)."""
    import torch
    from paper_1510_00561_amd import ct
    y = planes[0::3]
    cur, prev = y[1:].contiguous(), y[:-1].contiguous()
    mv, ssd = ct.motion_search(cur, prev, w)
    torch.cuda.synchronize()
    ct.profile_enable(True, 1024)
    for _ in range(steps):
        ct.motion_search(cur, prev, w, mv, ssd)
    torch.cuda.synchronize()
    stats = ct.profile_collect()
    ct.profile_enable(False)
    cnt, tms, by = stats["motion_search"]
    B, Hh, Ww = cur.shape
    evals = B * (2 * w + 1) ** 2 * Hh * Ww          # candidate pixels per launch
    us = tms / cnt * 1e3
    rate = evals / (us * 1e-6)
    return {"workload": f"{B} pairs of consecutive {Ww}x{Hh} Y planes, 16x16 blocks, w={w} "
                        f"({(2 * w + 1) ** 2} candidates)",
            "avg_launch_us": round(us, 2), "pairs_per_s": round(B / (us * 1e-6), 1),
            "roofline": {"bound": "alu", "achieved": round(rate / 1e12, 3), "peak": VALU_LANE_OPS / 1e12,
                         "unit": "T candidate-pixels/s", "frac": round(rate / VALU_LANE_OPS, 4),
                         "traffic": measured_traffic("motion_search", by / cnt, "traffic_motion_1080p.json"),
                         "compulsory_bytes": by / cnt},
            "moving_blocks": int((mv != 0).any(dim=-1).sum())}


def batched_comparison(steps):
    """Mixed workload: 64 streams (one YCoCg frame each) of 320x240, 640x480 or
    1280x720, LP depth 2-4, 8-16 directions, as one graph launch of grouped
    kernels vs the same work as per-stream, per-stage plain launches."""
    import numpy as np
    import torch
    from paper_1510_00561_amd import ct, synth
    streams = synth.mixed_streams(64, 4)
    clips = {}
    for (h, w) in sorted({(s[0], s[1]) for s in streams}):
        clips[(h, w)] = ycocg_planes(torch.from_numpy(synth.clip_rgb(8, h, w, 4)).cuda())
    rng = synth.rng_for(4)
    descs = []
    for i, (h, w, J, dirs) in enumerate(streams):
        fr = i % 8
        planes = clips[(h, w)][3 * fr:3 * fr + 3].contiguous()
        nsub = int(ct.layout(h, w, J, dirs)[0].nsub)
        step_table = torch.from_numpy(rng.integers(4, 65, size=(3, nsub)).astype(np.float32)).cuda()
        descs.append(dict(height=h, width=w, levels=J, dirs=dirs, planes=planes, steps=step_table))
    plan = ct.Batched(descs, graph=True, autotune=True, fused=True)
    plan.run()
    plan.run_plain()
    torch.cuda.synchronize()
    ref = [s["out"].clone() for s in plan.streams]
    plan.run()
    torch.cuda.synchronize()
    identical = all(torch.equal(a, s["out"]) for a, s in zip(ref, plan.streams))
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    t_plain = timed(plan.run_plain)
    t_graph = timed(plan.run)
    info = plan.info()
    plan.close()
    return {"workload": "64 streams (one YCoCg frame each) drawn from 320x240/640x480/1280x720, "
                        "LP depth 2-4, 8-16 directions, fused encoder + decoder",
            "t_plain_ms": round(t_plain, 3), "t_batched_graph_ms": round(t_graph, 3),
            "speedup": round(t_plain / t_graph, 3), "frames_per_s_batched": round(64 / (t_graph / 1e3), 1),
            "bit_identical_to_plain": identical, "plan": info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip timing the four separate calls (profiling runs)")
    ap.add_argument("--mode", choices=["bench", "copy", "colour", "motion"], default="bench",
                    help="copy: stream 1 GiB through a plain elementwise kernel (counter calibration); "
                         "colour: only the colour and K-frame stages, --steps launches of each; "
                         "motion: only the motion search, --steps launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1510_00561_amd import ct, synth

    if args.mode == "copy":
        n = 1 << 28                                   # 2^28 floats = 1 GiB each way
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                          "launches": args.steps}))
        return

    if args.mode == "motion":
        rgb = torch.from_numpy(synth.clip_rgb(FRAMES, H, W, 3)).to("cuda:0")
        print(json.dumps({"mode": "motion", "motion": motion_stage(ycocg_planes(rgb), args.steps)}))
        return

    if args.mode == "colour":
        # the colour and K-frame stages alone, every launch at chroma factor 4
        # (for their kernel traces and counters); the lowpass indices come
        # from the 16 Y planes, each encoded three times
        rgb = torch.from_numpy(synth.clip_rgb(FRAMES, H, W, 3)).to("cuda:0")
        plan = ct.Plan(H, W, J, DIRS, PLANES, "cuda:0")
        steps_tab = synth.subband_steps(plan.nsub, 3, 3)
        steps = torch.from_numpy(np.stack([steps_tab[b % 3] for b in range(PLANES)])).to("cuda:0")
        y4, _, _ = ct.rgb_to_ycocg(rgb, 4)
        idx, _ = plan.encode(y4.repeat(3, 1, 1).contiguous(), steps)
        fb = front_back_stages(rgb, plan, idx, args.steps, check_factor1=False)
        print(json.dumps({"mode": "colour", "front_back": fb}))
        return

    print(f"[bench] generating {FRAMES} frames of {W}x{H}", file=sys.stderr, flush=True)
    rgb_np = synth.clip_rgb(FRAMES, H, W, 3)
    plan = ct.Plan(H, W, J, DIRS, PLANES, "cuda:0")
    steps_tab = synth.subband_steps(plan.nsub, 3, 3)            # [3][nsub]
    steps_np = np.stack([steps_tab[b % 3] for b in range(PLANES)]).astype(np.float32)

    dev = torch.device("cuda:0")
    rgb = torch.from_numpy(rgb_np).to(dev)
    x = ycocg_planes(rgb)
    steps = torch.from_numpy(steps_np).to(dev)
    coef = torch.empty((PLANES, plan.ncoef), dtype=torch.float32, device=dev)
    coef2 = torch.empty_like(coef)
    idx = torch.empty((PLANES, plan.ncoef), dtype=torch.int16, device=dev)
    side = torch.empty((PLANES, 2), dtype=torch.float32, device=dev)
    rec = torch.empty_like(x)

    idx2 = torch.empty_like(idx)
    side2 = torch.empty_like(side)
    rec2 = torch.empty_like(x)

    def step():
        # the codec step: fused encoder (forward CT + quantise) and decoder
        # (dequantise + inverse CT)
        plan.encode(x, steps, idx, side)
        plan.decode(idx, steps, side, out=rec)

    def step_separate():
        # the same step as four separate calls, with float coefficients in HBM
        plan.forward(x, out=coef)
        plan.quantize(coef, steps, idx2, side2)
        plan.dequantize(idx2, steps, side2, out=coef2)
        plan.inverse(coef2, out=rec2)

    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, time.perf_counter() - t0

    ms_sep = None
    if not args.no_separate:
        ms_sep, _ = timed(step_separate)
    ms, wall = timed(step)
    identical = None
    if ms_sep is not None:
        identical = bool(torch.equal(idx, idx2) and torch.equal(side, side2) and torch.equal(rec, rec2))
    err = float((rec - x).abs().max())

    alg = algorithmic_bytes_per_plane(plan.ncoef) * PLANES
    fps = FRAMES / (ms / 1e3)
    eff_gbps = alg / (ms / 1e3) / 1e9

    roofline = None
    kernels = {}
    if not args.no_profile:
        ct.profile_enable(True, 8192)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        stats = ct.profile_collect()
        ct.profile_enable(False)
        total = sum(v[1] for v in stats.values())
        for name, (n, tms, by) in stats.items():
            kernels[name] = {"launches_per_step": n / args.steps, "ms_per_step": tms / args.steps,
                             "share": tms / total if total else 0.0,
                             "gbps": by / (tms / 1e3) / 1e9 if tms else 0.0}
        dom = max(stats.items(), key=lambda kv: kv[1][1])
        name, (n, tms, by) = dom
        achieved = by / (tms / 1e3) / 1e9
        traffic = measured_traffic(name, by / n)
        roofline = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic, "avg_launch_us": round(tms / n * 1e3, 2),
                    "bytes_per_launch": by / n}

    batched = None
    if not args.no_batched:
        print("[bench] batched mixed-stream comparison", file=sys.stderr, flush=True)
        batched = batched_comparison(max(3, args.steps // 2))

    print("[bench] colour and K-frame stages", file=sys.stderr, flush=True)
    fb = front_back_stages(rgb, plan, idx, max(3, args.steps // 2))
    print("[bench] motion search", file=sys.stderr, flush=True)
    me = motion_stage(x, max(3, args.steps // 2))

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(rgb_np[0], steps_tab)

    out = {
        "metric": METRIC, "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "16 x 1920x1080 YCoCg frames (48 planes, padded 1088x1920), "
                               "CT J=4 dirs 32/16/8/8, forward+quantise (fused encoder) then "
                               "dequantise+inverse (fused decoder), per-subband steps 4..64",
                   "frames": FRAMES, "planes": PLANES, "levels": J, "dirs": DIRS},
        "hbm_effective_gbps": round(eff_gbps, 1),
        "hbm_effective_frac": round(eff_gbps / HBM_PEAK_GBPS, 4),
        "algorithmic_bytes_per_step": alg,
        "roundtrip_max_abs_err": err,
        "separate_calls_ms_per_step": round(ms_sep, 4) if ms_sep else None,
        "fused_speedup_vs_separate": round(ms_sep / ms, 3) if ms_sep else None,
        "fused_bit_identical_to_separate": identical,
        "wall_s": round(wall, 3),
        "roofline": roofline,
        "kernels": kernels,
        "batched": batched,
        "front_back": fb,
        "motion": me,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
