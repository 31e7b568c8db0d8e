"""The quantiser's index functions on the host (no GPU): the select-form
rounding of to_index against rounding halves away from zero on doubles, and
the reciprocal-based quotient of quant_index against the correctly rounded
division, on steps and values that stress both (tests/host/quant_index.cpp
includes ct_quant_stages.h itself, so the code under test is the library's)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    return shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.mark.skipif(_hipcc() is None, reason="hipcc is needed to build the host harness")
def test_quant_index_matches_the_division(tmp_path):
    exe = str(tmp_path / "quant_index")
    cmd = [_hipcc(), "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-ffp-contract=off",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1510_00561_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "quant_index.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-2000:]
    assert "quant index clean" in run.stdout
