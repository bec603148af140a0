"""Host-side logic of the benchmark (no GPU): the algorithmic operation count
behind the k-step kernel's roofline, the one-GPU guard and the CPU baseline."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_op_count_per_cell_update():
    # 8 vmax per 32-cell word for rules 1-4 and F(t); 44 more when p draws
    assert bench.kstep_ops_per_cell_update(0, 0.0) == 0.0
    assert bench.kstep_ops_per_cell_update(5, 0.0) == 40 / 32
    assert bench.kstep_ops_per_cell_update(5, 0.13) == (40 + 44) / 32
    assert bench.kstep_ops_per_cell_update(8, 0.5) == (64 + 44) / 32
    # thr = floor(p 2^32) = 0: rule 3 never fires and nothing is drawn
    assert bench.kstep_ops_per_cell_update(3, 2.0 ** -33) == 24 / 32
    assert bench.kstep_ops_per_cell_update(3, 2.0 ** -32) == (24 + 44) / 32


def test_alu_peak_from_unit_counts():
    assert bench.VALU_PEAK == pytest.approx(39.3216e12)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "--gpus 1" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_reports_all_core_and_serial_oracle():
    from paper_2309_14311_amd import workloads
    reps = workloads.ensemble(8, seed=1, T=5000, warmup=1000)
    cb = bench.cpu_baseline_ensemble(reps, budget_s=0.2, steps=10)
    assert cb["kind"] == "oracle" and cb["unit"] == "cell-updates/s"
    assert cb["value"] > 0 and 1 <= cb["cores"] <= 16
    assert cb["serial"]["cores"] == 1 and cb["serial"]["value"] > 0
    assert "replicas" in cb["sample"] and "replicas" in cb["serial"]["sample"]


@pytest.mark.parametrize("name,rng", [("LARGE_RING", "keyed"), ("OPEN_ROAD", "keyed"),
                                      ("AGENT_RING", "stream"), ("REFERENCE", "keyed")])
def test_cpu_baseline_of_one_road_workloads(name, rng):
    from paper_2309_14311_amd import workloads
    cb = bench.cpu_baseline_single(getattr(workloads, name), budget_s=0.05, rng=rng,
                                   max_cells=1 << 14)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["serial"]["value"] > 0
    assert cb["cores"] >= 1 and cb["serial"]["cores"] == 1
    assert cb["host"]["logical_cpus"] >= 1
