"""The byte <-> bit-plane conversions of the bit-sliced kernels (bitplanes.hpp),
built for the host with a model of the device's byte permute and checked
against cell-by-cell definitions: the 4 x 4 byte transpose, the code planes and
occupancy of random road words and their round trip, and the thermometer
planes of every vmax (0xFF empty, else v <= vmax) with their way back to
bytes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not found")
def test_bitplane_conversions(tmp_path):
    exe = str(tmp_path / "bitplanes_check")
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "paper_2309_14311_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "bitplanes_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
