"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the colour stages' per-thread indexing (tests/host/color_bounds.cpp runs every
thread of each launch shape over exactly sized buffers) and the codec's host
entry points (tests/host/codec_fuzz.cpp: the zero-run decoder and DEFLATE on
valid and corrupted streams)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    return shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.mark.skipif(_hipcc() is None, reason="hipcc is needed to build the host harness")
def test_colour_stage_indexing_is_sanitizer_clean(tmp_path):
    exe = str(tmp_path / "color_bounds")
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        san += ["-Xarch_host", flag]     # host code only
    cmd = [_hipcc(), "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17"] + san + [
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1510_00561_amd", "csrc"),
        os.path.join(ROOT, "tests", "host", "color_bounds.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, (run.stdout + run.stderr)[-2000:]
    assert "shapes clean" in run.stdout


@pytest.mark.skipif(_hipcc() is None, reason="hipcc is needed to build the host harness")
def test_codec_host_entry_points_are_sanitizer_clean(tmp_path):
    exe = str(tmp_path / "codec_fuzz")
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        san += ["-Xarch_host", flag]     # host code only
    cmd = [_hipcc(), "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17"] + san + [
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1510_00561_amd", "csrc"),
        os.path.join(ROOT, "tests", "host", "codec_fuzz.cpp"), "-o", exe, "-lz"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-2000:]
    assert "codec host entry points clean" in run.stdout
