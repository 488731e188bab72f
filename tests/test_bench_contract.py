"""The bench.py command-line contract.

* More than one GPU is refused up front, with a message and a nonzero exit,
  before anything touches a GPU (CPU test).
* A short run of the default workload prints exactly one JSON line on stdout
  carrying the fields the measurement record needs: the metric and its unit,
  whole-job value, step timing, the workload, the live roofline of the
  dominant kernel and its HBM traffic record (GPU test).
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, timeout=600):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2", timeout=120)
    assert r.returncode == 2
    assert r.stdout == ""
    assert "one GPU" in r.stderr


def one_line(r):
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 0
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert "workload" in d["config"]
    roof = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in roof, key
    assert 0.0 < roof["frac"] <= 1.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-12
    return d


@pytest.mark.gpu
def test_default_bench_prints_one_json_line():
    # the default workload (n = 4000 completion), cut to one step and no solves
    r = run_bench("--steps", "1", "--warmup", "0", "--no-cpu-baseline", "--no-config1", "--solve", "",
                  "--forms", "f64,f64_sampled", "--form-loop", "3")
    d = one_line(r)
    assert "n=4000" in d["config"]["workload"]
    roof = d["roofline"]
    assert roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s" and roof["peak"] == 78.6
    # the sampled kernels are reported at algorithmic HBM bytes: never above the peak
    for key in ("sampled_ye", "sampled_dots"):
        assert 0.0 < d["forms"]["f64_sampled"][key]["frac"] <= 1.0, key


@pytest.mark.gpu
def test_sensing_bench_prints_one_json_line():
    r = run_bench("--workload", "sensing", "--steps", "1", "--warmup", "0", "--no-cpu-baseline", "--no-mixed",
                  "--apply-loop", "10")
    d = one_line(r)
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
