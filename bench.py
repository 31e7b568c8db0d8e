"""Benchmark: contourlet forward + quantise + dequantise + inverse on 1080p frames.

One step is the whole hot path on one batch: 16 synthetic 1920x1080 RGB
frames, converted to YCoCg by the library beforehand (48 float32 planes: Y,
Co + 127, Cg + 127, padded to 1088 x 1920), LP 4 levels,
DFB 32/16/8/8 directions, per-subband quantisation steps drawn per channel
from 4..64. Inputs are resident in HBM before timing starts.

Prints one JSON line. `value` is frames/s (real 1080p frames). The line also
carries the effective HBM bandwidth of the step (algorithmic bytes / time),
the roofline of the dominant kernel from live per-launch HIP events, the
colour front end / back end, the K-frame lowpass filter, the motion search and
the codec back end (P-frame components, zero-run coding, DEFLATE) measured on
the same frames (outside the step), a copy kernel as the attainable ceiling,
and the FP64 oracle timed on the host cores on a bounded sample.
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
    "dfb_split3_analysis": ("ct_level.hip", "ct_stream.h", "ct_stages.h", "ct_kernels.h", "ct_api.cpp"),
    "dfb_split3_synthesis": ("ct_level.hip", "ct_stream.h", "ct_stages.h", "ct_kernels.h", "ct_api.cpp"),
    "pad_fold": ("ct_level.hip",),
    "lowpass_partial": ("ct_quant.hip", "ct_quant_stages.h"),
    "quantize": ("ct_quant.hip", "ct_quant_stages.h"),
    "dequantize": ("ct_quant.hip", "ct_quant_stages.h"),
    "rgb_to_ycocg": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "ycocg_to_rgb": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "lowpass_diff": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "lowpass_undiff": ("ct_color.hip", "ct_color_stages.h", "ct_color_api.cpp"),
    "motion_search": ("ct_motion.hip", "ct_motion.h", "ct_motion_api.cpp"),
    "mc_residual": ("ct_codec.hip", "ct_codec.h", "ct_codec_api.cpp"),
    "rle_encode": ("ct_codec.hip", "ct_codec.h", "ct_codec_api.cpp"),
}


def algorithmic_bytes_per_plane(ncoef):
    """Forward 4HW + 4n, quantise 4n + 2n, dequantise 2n + 4n, inverse 4n + 4HW."""
    return 8 * H * W + 20 * ncoef


def _with_includes(files):
    """The files and every local header they include, transitively, in a
    fixed order."""
    csrc = os.path.join(ROOT, "paper_1510_00561_amd", "csrc")
    seen, todo = [], list(files)
    while todo:
        fn = todo.pop(0)
        if fn in seen or not os.path.exists(os.path.join(csrc, fn)):
            continue
        seen.append(fn)
        with open(os.path.join(csrc, fn)) as f:
            for line in f:
                line = line.strip()
                if line.startswith('#include "') and "/" not in line:
                    todo.append(line.split('"')[1])
    return seen


def source_digest(name):
    """Digest of a kernel's sources (with the headers they include): a counter
    summary taken from other sources is stale."""
    h = hashlib.sha256()
    for fn in _with_includes(KERNEL_SOURCES.get(name, ())):
        with open(os.path.join(ROOT, "paper_1510_00561_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(name, bytes_per_launch=None, summary="traffic_1080p.json"):
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


def _oracle_plane(args):
    """One plane through the FP64 oracle: forward, quantise, dequantise, inverse."""
    import numpy as np
    from oracle import ct as oct
    from oracle import geometry as geo
    from oracle import quant as oq
    x, steps = args
    table = geo.subband_table(H, W, J, DIRS)
    c = oct.forward(np.asarray(x, np.float64), J, DIRS)
    q, side = oq.quantize64(c, np.asarray(steps, np.float64), table)
    d = oq.dequantize64(q, np.asarray(steps, np.float64), side, table)
    oct.inverse(d, H, W, J, DIRS)
    return 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rgb_frames, steps_np, workers=None):
    """The FP64 oracle on the host cores: one plane in one process (latency),
    then a process pool over up to three planes per worker (throughput)."""
    import multiprocessing as mp
    import numpy as np
    from oracle import color
    planes = [p for fr in rgb_frames for p in color.encode_frame(fr, 1)]
    jobs = [(planes[i], steps_np[i % 3]) for i in range(len(planes))]
    t0 = time.perf_counter()
    _oracle_plane(jobs[0])
    latency = time.perf_counter() - t0
    # at most 16 worker processes (a share of a large host), one per core below that
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    n = min(len(jobs), 3 * workers)
    ctx = mp.get_context("spawn")
    # one thread per worker process: the pool, not the math libraries, uses
    # the cores (spawned workers take the environment at start)
    thread_vars = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {v: os.environ.get(v) for v in thread_vars}
    for v in thread_vars:
        os.environ[v] = "1"
    try:
        with ctx.Pool(workers) as pool:
            pool.map(_oracle_plane, jobs[:workers])          # start-up and first-touch, untimed
            t0 = time.perf_counter()
            pool.map(_oracle_plane, jobs[:n])
            dt = time.perf_counter() - t0
    finally:
        for v, val in saved.items():
            if val is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = val
    return {"value": round(n / 3.0 / dt, 4), "unit": "frames/s", "cores": workers, "kind": "oracle",
            "cpu": cpu_model(), "threads_per_process": 1,
            "single_plane_latency_s": round(latency, 2),
            "single_process_frames_per_s": round(1.0 / 3.0 / latency, 4),
            "sample": f"{n} planes (Y, Co, Cg of {n // 3} 1080p frames) forward+quantise+dequantise+inverse "
                      f"in FP64 NumPy over a pool of {workers} processes ({dt:.1f} s); latency of one "
                      f"plane in one process {latency:.1f} s"}


def tuned_shapes():
    """The split-pass tile shapes the tuner chose for the 1080p levels, from
    its cache file: {level shape: (tree levels per pass, block height)}."""
    path = os.environ.get("CT_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                                 "ct_autotune.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        entries = json.load(f)
    out = {}
    for key, code in entries.items():
        parts = key.split("|")
        if len(parts) != 5 or parts[1] != "split_tune" or parts[4] != f"b{PLANES}":
            continue
        rows, cols = (int(v) for v in parts[2].split("x"))
        if (rows, cols) not in [((H + 15) // 16 * 16 >> j, W >> j) for j in range(J)]:
            continue
        mode = (code >> 4) & 3
        height = ["default", "short", "tall", f"{((code >> 8) & 255) * 4} rows"][mode]
        out[f"{parts[2]} {parts[3]}"] = {"levels_per_pass": code & 15, "block_height": height}
    return out


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


def copy_ceiling(steps):
    """Attainable bandwidth: a plain streaming copy (read + write, 1 GiB each way)
    timed with HIP events on the current stream."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gbps = 8.0 * n / (ms * 1e-3) / 1e9
    del a, b
    return {"kernel": "torch.mul(a, 1.0, out=b) over 2^28 floats", "bytes_per_launch": 8 * n,
            "avg_launch_us": round(ms * 1e3, 2), "gbps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4)}


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
    ct.profile_enable(True, 64)
    plan.run()
    torch.cuda.synchronize()
    stats = ct.profile_collect(alg=True)
    ct.profile_enable(False)
    _, _, comp_b, alg_b = stats["batched_graph"]
    info = plan.info()
    plan.close()
    return {"workload": "64 streams (one YCoCg frame each) drawn from 320x240/640x480/1280x720, "
                        "LP depth 2-4, 8-16 directions, fused encoder + decoder",
            "t_plain_ms": round(t_plain, 3), "t_batched_graph_ms": round(t_graph, 3),
            "speedup": round(t_plain / t_graph, 3), "frames_per_s_batched": round(64 / (t_graph / 1e3), 1),
            "alg_bytes_per_run": alg_b, "compulsory_bytes_per_run": comp_b,
            "hbm_alg_gbps": round(alg_b / (t_graph * 1e-3) / 1e9, 1),
            "hbm_alg_frac": round(alg_b / (t_graph * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "hbm_compulsory_frac": round(comp_b / (t_graph * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "bit_identical_to_plain": identical, "plan": info}


def codec_back_end(plan, x, steps, reps):
    """The codec stages after the quantiser on the step's 16 frames: frame 0 is a
    K-frame, frames 1..15 P-frames (vectors from the motion search on the Y
    planes, w = 8). Device times of the P-frame components and the zero-run
    coder; DEFLATE (host) on the first K-frame and the first P-frame gives the
    coded size."""
    import numpy as np
    import torch
    from paper_1510_00561_amd import ct
    idx, side = plan.encode(x, steps)
    B = x.shape[0]
    y = x[0::3]
    mv, _ = ct.motion_search(y[1:].contiguous(), y[:-1].contiguous(), 8)
    pl = ct.Plan(H, W, J, DIRS, B - 3, "cuda:0")
    cur, prev = idx[3:].contiguous(), idx[:-3].contiguous()
    res = pl.mc_residual(cur, prev, mv, n=1, group=3)
    pk = ct.Plan(H, W, J, DIRS, 3, "cuda:0")
    k_sym, k_off = pk.rle_encode(idx[:3].contiguous(), 0)
    p_sym, p_off = pl.rle_encode(res, 1)
    back = pl.mc_residual(res, prev, mv, n=1, group=3, inverse=True)
    torch.cuda.synchronize()
    restored = bool(torch.equal(back, cur))
    ct.profile_enable(True, 1024)
    for _ in range(reps):
        pl.mc_residual(cur, prev, mv, n=1, group=3, out=res)
        pl.rle_encode(res, 1, p_sym, p_off)
    torch.cuda.synchronize()
    stats = ct.profile_collect(alg=True)
    ct.profile_enable(False)
    dev = {}
    for name, (n, tms, by, al) in stats.items():
        us = tms / n * 1e3
        dev[name] = {"avg_launch_us": round(us, 2), "bytes_per_launch": by / n,
                     "gbps": round(by / n / (us * 1e3), 1), "frac": round(by / n / (us * 1e3) / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic(name, by / n, "traffic_codec_1080p.json")}
    k_sym_h, k_off_h = k_sym.cpu().numpy(), k_off.cpu().numpy()
    p_sym_h, p_off_h = p_sym.cpu().numpy(), p_off.cpu().numpy()
    sizes = {}
    t0 = time.perf_counter()
    for kind, symh, offh, planes in (("k_frame", k_sym_h, k_off_h, range(3)), ("p_frame", p_sym_h, p_off_h, range(3))):
        tot_scal, tot_nts, syms = 0, 0, 0
        for b in planes:
            s_b = symh[b, :offh[b, -1]]
            blob, _ = ct.deflate_host(s_b, offh[b], 0)
            blob1, _ = ct.deflate_host(s_b, offh[b], 1)
            tot_scal += len(blob)
            tot_nts += len(blob1)
            syms += int(offh[b, -1])
        sizes[kind] = {"symbols": syms, "bytes_scalable": tot_scal, "bytes_nts": tot_nts,
                       "bits_per_pixel_scalable": round(8.0 * tot_scal / (H * W), 4),
                       "bits_per_pixel_nts": round(8.0 * tot_nts / (H * W), 4)}
    deflate_s = time.perf_counter() - t0
    del pl, pk
    return {"workload": f"{B // 3} YCoCg 1080p frames: frame 0 a K-frame, frames 1..{B // 3 - 1} P-frames "
                        f"(motion search w=8 on Y, vectors shared by the three channels)",
            "kernels": dev, "p_frames_restored_exactly": restored,
            "deflate_host_s_for_two_frames": round(deflate_s, 3), "sizes_first_frames": sizes}


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
    ap.add_argument("--no-tune", action="store_true",
                    help="run the step with the default tile shapes (no ct_autotune)")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the step only: no colour, motion or codec stages (counter runs)")
    ap.add_argument("--mode", choices=["bench", "copy", "colour", "motion", "codec"], default="bench",
                    help="copy: stream 1 GiB through a plain elementwise kernel (counter calibration); "
                         "colour: only the colour and K-frame stages, --steps launches of each; "
                         "motion: only the motion search, --steps launches; "
                         "codec: only the P-frame components and the zero-run coder, --steps launches")
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

    if args.mode == "codec":
        rgb = torch.from_numpy(synth.clip_rgb(FRAMES, H, W, 3)).to("cuda:0")
        plan = ct.Plan(H, W, J, DIRS, PLANES, "cuda:0")
        steps_tab = synth.subband_steps(plan.nsub, 3, 3)
        steps = torch.from_numpy(np.stack([steps_tab[b % 3] for b in range(PLANES)])).to("cuda:0")
        print(json.dumps({"mode": "codec", "codec": codec_back_end(plan, ycocg_planes(rgb), steps, args.steps)}))
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

    # tile shapes of the split passes, tuned once for this shape (outside the
    # timed region; the choice does not change a bit of the output)
    tuned = None
    if not args.no_tune:
        t0 = time.perf_counter()
        plan.autotune()
        tuned = {"seconds": round(time.perf_counter() - t0, 2), "levels": tuned_shapes()}

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
    step_traffic = None
    fused_bytes = None
    if not args.no_profile:
        # per-launch times of each kernel on its own: the profiled steps run
        # the chain in order on one stream (the timed steps above overlap the
        # level-1 passes with the coarse levels, which stretches both)
        os.environ["CT_SERIAL_LEVELS"] = "1"
        ct.profile_enable(True, 8192)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        stats = ct.profile_collect(alg=True)
        ct.profile_enable(False)
        del os.environ["CT_SERIAL_LEVELS"]
        total = sum(v[1] for v in stats.values())
        fused_bytes = sum(v[3] for v in stats.values()) / args.steps
        step_traffic = 0.0
        for name, (n, tms, by, al) in stats.items():
            us = tms / n * 1e3
            tr = measured_traffic(name)
            if tr is None:
                step_traffic = None
            elif step_traffic is not None:
                step_traffic += tr * n / args.steps
            kernels[name] = {"launches_per_step": n / args.steps, "ms_per_step": round(tms / args.steps, 4),
                             "share": round(tms / total, 4) if total else 0.0, "avg_launch_us": round(us, 2),
                             "alg_bytes_per_launch": al / n, "compulsory_bytes_per_launch": by / n,
                             "alg_gbps": round(al / n / (us * 1e3), 1), "compulsory_gbps": round(by / n / (us * 1e3), 1),
                             "frac_alg": round(al / n / (us * 1e3) / HBM_PEAK_GBPS, 4),
                             "frac_compulsory": round(by / n / (us * 1e3) / HBM_PEAK_GBPS, 4),
                             "traffic_bytes_per_launch": tr,
                             "traffic_over_compulsory": round(tr / (by / n), 3) if tr else None}
        dom = max(stats.items(), key=lambda kv: kv[1][1])
        name, (n, tms, by, al) = dom
        us = tms / n * 1e3
        achieved = al / n / (us * 1e3)           # algorithmic bytes per launch / launch time, GB/s
        roofline = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": measured_traffic(name), "avg_launch_us": round(us, 2),
                    "alg_bytes_per_launch": al / n, "compulsory_bytes_per_launch": by / n,
                    "compulsory_achieved": round(by / n / (us * 1e3), 1),
                    "compulsory_frac": round(by / n / (us * 1e3) / HBM_PEAK_GBPS, 4)}

    copy = None if args.no_extras else copy_ceiling(max(5, args.steps // 2))

    batched = None
    if not args.no_batched:
        print("[bench] batched mixed-stream comparison", file=sys.stderr, flush=True)
        batched = batched_comparison(max(3, args.steps // 2))

    variants = None
    if not args.no_extras:
        # the same fused step with the variant filter pair and reconstruction
        print("[bench] variant filters and reconstruction", file=sys.stderr, flush=True)
        variants = {}
        for f, r in (("53", "dual"), ("97", "ba"), ("53", "ba")):
            vp = ct.Plan(H, W, J, DIRS, PLANES, "cuda:0", filters=f, recon=r)
            vrec = torch.empty_like(x)

            def vstep():
                vp.encode(x, steps, idx2, side2)
                vp.decode(idx2, steps, side2, out=vrec)
            vms, _ = timed(vstep)
            variants[f"{f}_{r}"] = {"filters": {"97": "CDF 9-7", "53": "LeGall 5/3"}[f],
                                    "recon": {"dual": "dual frame", "ba": "Burt-Adelson"}[r],
                                    "ms_per_step": round(vms, 4), "frames_per_s": round(FRAMES / (vms / 1e3), 1),
                                    "roundtrip_max_abs_err": float((vrec - x).abs().max())}
            del vp, vrec

    rgb_enc = None
    if not args.no_extras:
        # the encoder from the 8-bit frames: colour transform fused into the
        # first LP level's loads, against the colour kernel + plane stacking
        # + fused encoder
        print("[bench] RGB encoder", file=sys.stderr, flush=True)

        def enc_rgb():
            plan.encode_rgb(rgb, steps, idx2, side2)

        def enc_sep():
            plan.encode(ycocg_planes(rgb), steps, idx, side)
        ms_f, _ = timed(enc_rgb)
        ms_s, _ = timed(enc_sep)
        rgb_enc = {"workload": f"{FRAMES} RGB frames {W}x{H} -> indices of {PLANES} planes",
                   "ms_fused": round(ms_f, 4), "ms_colour_then_encode": round(ms_s, 4),
                   "frames_per_s_fused": round(FRAMES / (ms_f / 1e3), 1),
                   "identical": bool(torch.equal(idx, idx2) and torch.equal(side, side2))}
        plan.encode(x, steps, idx, side)      # the step's indices again, for the stages below

    fb = me = codec = None
    if not args.no_extras:
        print("[bench] colour and K-frame stages", file=sys.stderr, flush=True)
        fb = front_back_stages(rgb, plan, idx, max(3, args.steps // 2))
        print("[bench] motion search", file=sys.stderr, flush=True)
        me = motion_stage(x, max(3, args.steps // 2))
        print("[bench] codec back end", file=sys.stderr, flush=True)
        codec = codec_back_end(plan, x, steps, max(3, args.steps // 2))

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(rgb_np, steps_tab)

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
        "fused_compulsory_bytes_per_step": fused_bytes,
        "fused_compulsory_frac": round(fused_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4) if fused_bytes else None,
        "counter_traffic_bytes_per_step": step_traffic,
        "traffic_over_alg": round(step_traffic / alg, 3) if step_traffic else None,
        "traffic_over_fused_compulsory": round(step_traffic / fused_bytes, 3) if step_traffic and fused_bytes else None,
        "copy_ceiling": copy,
        "hbm_effective_over_copy": round(eff_gbps / copy["gbps"], 4) if copy else None,
        "roundtrip_max_abs_err": err,
        "separate_calls_ms_per_step": round(ms_sep, 4) if ms_sep else None,
        "fused_speedup_vs_separate": round(ms_sep / ms, 3) if ms_sep else None,
        "fused_bit_identical_to_separate": identical,
        "tile_shapes": tuned,
        "wall_s": round(wall, 3),
        "roofline": roofline,
        "kernels": kernels,
        "batched": batched,
        "variants": variants,
        "rgb_encoder": rgb_enc,
        "front_back": fb,
        "motion": me,
        "codec": codec,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
