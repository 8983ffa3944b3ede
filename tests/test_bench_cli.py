"""The bench's command line: one JSON line with the contract's fields (GPU),
and the refusal of more than one GPU (CPU).  The GPU case runs the bench in
a child process with short settings and a 64-receiver oracle sample."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2", timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_bench_json_line():
    r = _bench("--steps", "2", "--warmup", "1", "--secondary", "0", "--cpu-frames", "2", "--cpu-rx", "8",
               timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["dtype"] == "f32" and d["data"] == "synthetic"
    assert d["config"]["workload"].startswith("crowd") and d["config"]["frames"] == 256
    # throughput = (rx x body x freq) evaluations per step over the step time
    ev = d["config"]["evals_per_step"]
    assert abs(d["value"] - ev / (d["ms_per_step"] * 1e-3)) <= 1e-6 * d["value"]
    rf = d["roofline"]
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    assert 0.0 < rf["frac"] < 1.0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    assert rf["kernel_ms"] <= d["ms_per_step"] * 1.05
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and "2 crowd frames" in cb["sample"]
    assert cb["fp32_field_error"]["max_normwise_rel"] <= 1e-4
