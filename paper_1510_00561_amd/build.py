"""Builds libct.so (HIP for gfx950) in-tree with hipcc.

The library lands next to this file as `libct.so`; the ctypes binding loads
it from there. Every source is compiled for gfx950 only, with packed FP32
instructions disabled. The quantiser translation unit is built without FMA
contraction so that its float32 operation order is exactly the documented one.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libct.so")

SOURCES = [
    ("ct_geometry.cpp", []),
    ("ct_filters.cpp", []),
    ("ct_api.cpp", []),
    ("ct_plan.cpp", []),
    ("ct_tune.cpp", []),
    ("ct_level.hip", ["-ffp-contract=off"]),
    ("ct_quant.hip", ["-ffp-contract=off"]),
    ("ct_batched.hip", ["-ffp-contract=off"]),
    ("ct_color_api.cpp", []),
    ("ct_color.hip", ["-ffp-contract=off"]),
    ("ct_motion_api.cpp", []),
    ("ct_motion.hip", []),
    ("ct_noalloc.hip", []),
    ("ct_codec_api.cpp", []),
    ("ct_codec.hip", []),
]

COMMON = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-result",
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP toolchain is required to build libct")
    return path


def _compile(src, extra):
    out = os.path.join(BUILD_DIR, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [hipcc()] + lang + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return out


def build(verbose=False):
    """Compile every source and link libct.so; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lz"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
