"""Host-side logic of the benchmark (no GPU): the algorithmic operation count
behind the k-step kernel's roofline, the ALU peak's derivation, the one-GPU
guard and the CPU baseline's protocol (stratified sample, warm-up, median of
3 timed chunks)."""
import os
import subprocess
import sys
import time

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
    # 256 CU x 4 SIMD x 32 lanes x 2.4 GHz: half the 157.3 TFLOP/s fp32 vector
    # peak (an FMA counts two flops); 4-cycle instructions issue at half that
    assert bench.VALU_PEAK == pytest.approx(78.6432e12)
    assert bench.VALU_PEAK == pytest.approx(157.3e12 / 2, rel=1e-3)
    assert bench.VALU_PEAK_4CYCLE == pytest.approx(39.3216e12)


def test_stratified_sample_spans_every_size():
    reps = [dict(L=L) for L in (5, 1, 9, 3, 7, 2, 8, 4, 6, 10)]
    sample, m = bench._stratified(reps, 11)
    assert m == 5 and [r["L"] for r in sample] == [3, 8]
    sample, m = bench._stratified(reps, 1e9)        # never empty
    assert m == 1 and len(sample) == 10
    sample, m = bench._stratified(reps, 1)
    assert len(sample) == 1


def test_sample_descriptions_use_ordinals():
    assert [bench._ordinal(m) for m in (1, 2, 3, 4, 11, 12, 13, 21, 22, 23, 64, 101, 111)] == [
        "1st", "2nd", "3rd", "4th", "11th", "12th", "13th", "21st", "22nd", "23rd", "64th",
        "101st", "111th"]


def test_median_of_chunks_times_only_after_the_warm_up():
    calls = []

    def advance(t0, n):
        calls.append((t0, n))
        time.sleep(0.001 * n)

    rate, rates, warm, chunk = bench._median_of_chunks(advance, 100, 0.02, 0.01)
    # warm-up in doubling steps from t = 0, then three equal chunks continuing
    assert [n for _, n in calls[:-3]] == [2 ** i for i in range(len(calls) - 3)]
    assert warm == sum(n for _, n in calls[:-3]) and calls[-3][0] == warm
    assert [n for _, n in calls[-3:]] == [chunk] * 3 and chunk >= 1
    assert len(rates) == 3 and rate == sorted(rates)[1]


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
    cb = bench.cpu_baseline_ensemble(reps, 5000, budget_s=0.2)
    assert cb["kind"] == "oracle" and cb["unit"] == "cell-updates/s"
    assert cb["value"] > 0 and 1 <= cb["cores"] <= 16
    assert cb["serial"]["cores"] == 1 and cb["serial"]["value"] > 0
    assert "replicas" in cb["sample"] and "median of 3" in cb["sample"]
    assert cb["extrapolated"] is True and cb["extrapolated_full_workload_s"] > 0
    assert cb["omp"]["threads"] == cb["cores"]


@pytest.mark.parametrize("name,rng", [("LARGE_RING", "keyed"), ("OPEN_ROAD", "keyed"),
                                      ("AGENT_RING", "stream"), ("REFERENCE", "keyed")])
def test_cpu_baseline_of_one_road_workloads(name, rng):
    from paper_2309_14311_amd import workloads
    cfg = getattr(workloads, name)
    cb = bench.cpu_baseline_single(cfg, cfg["T"], budget_s=0.05, rng=rng, max_cells=1 << 14)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["serial"]["value"] > 0
    assert "median of 3" in cb["sample"] and cb["extrapolated"] is True
    assert cb["cores"] >= 1 and cb["serial"]["cores"] == 1
    assert cb["host"]["logical_cpus"] >= 1


def test_cpu_baseline_runs_in_a_child_with_cores_bound():
    """The benchmark times the oracle in a child process that starts its OpenMP
    runtime with OMP_PLACES=cores and OMP_PROC_BIND=spread, one thread per
    physical core."""
    from paper_2309_14311_amd import workloads
    cb = bench._cpu_baseline(dict(kind="single", cfg=workloads.REFERENCE, T=2000, budget=0.05,
                                  rng="keyed"))
    assert cb["omp"] == {"OMP_PLACES": "cores", "OMP_PROC_BIND": "spread",
                         "threads": bench._cpu_threads()}
    assert cb["value"] > 0 and cb["cores"] == bench._cpu_threads()
