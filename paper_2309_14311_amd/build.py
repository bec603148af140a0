"""Build libnasch.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed-FP32
instructions disabled, then linked into paper_2309_14311_amd/libnasch.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libnasch.so")

SOURCES = ["init.hip", "grid_kstep.hip", "grid_onestep.hip", "agent.hip", "runtime.hip",
           "batch.hip", "server.hip", "output.hip", "device_api.hip",
           "device_noalloc.hip"]
CLI_SRC = "traffic_main.cpp"
# measurement companion: the vector-ALU throughput probe (include/nasch_probe.h)
PROBE_SRC = "valu_probe.hip"
PROBE_LIB = os.path.join(PKG, "libnasch_probe.so")
CLI = os.path.join(PKG, "nasch_traffic")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # an LDS atomic that every lane of a wave issues on one address stays
          # one instruction (the step kernels reserve queue slots that way); the
          # default rewrites it into a scalar loop over the active lanes
          "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
          "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None) -> str:
    """Compile every HIP source and link libnasch.so; returns its path."""
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        raise RuntimeError("hipcc not found")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2) - 1), 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    pobj = _compile(PROBE_SRC)
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o",
                        PROBE_LIB + ".tmp", pobj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"probe link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    # the command-line driver, linked against the library next to it
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", INCLUDE, os.path.join(CSRC, CLI_SRC), "-o",
           CLI + ".tmp", "-L", PKG, "-lnasch", "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"nasch_traffic build failed:\n{r.stdout}\n{r.stderr}")
    os.replace(CLI + ".tmp", CLI)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))
