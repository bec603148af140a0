"""The runtime's tiling arithmetic (engine.hpp), built for the host and checked
against its definitions: the k-step tile geometry (halo a whole word and at
least k vmax, tiles covering the ring exactly, the largest admissible k), the
agent tiling, and the agent form's default cars per lane."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not found")
def test_tiling_arithmetic(tmp_path):
    exe = str(tmp_path / "engine_check")
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "paper_2309_14311_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "engine_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
