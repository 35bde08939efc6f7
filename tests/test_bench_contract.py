"""bench.py's command-line contract: one GPU only (a multi-GPU request exits
with a message before touching a device), and, on a GPU, one JSON line whose
fields carry the metric, the configuration, the roofline of the dominant
kernel and the measured copy ceiling."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          cwd=ROOT, capture_output=True, text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = run_bench("--gpus", "2", timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


@pytest.mark.gpu
def test_one_json_line_with_the_contract_fields():
    p = run_bench("--steps", "20", "--warmup", "2", "--no-cpu-baseline", "--no-variants")
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 2
    assert d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["value"] > 0 and d["ms_per_step"] > 0
    # whole-job throughput: nodes per step over the step time
    nodes = d["config"]["nodes"]
    assert abs(d["value"] - nodes / (d["ms_per_step"] * 1e-3) / 1e6) <= 1e-3 * d["value"]
    assert d["config"]["workload"].startswith("cylinder_heave_2048x4096")
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert 0 < r["frac"] < 1
    assert r["copy_ceiling"]["GBs"] > r["achieved"]
