"""bench.py end to end on a small instance of the headline workload: one JSON
line with the fields the measurement contract names (metric, value, roofline
with its peak and fraction, the kernels, the mode not used as headline)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("single", [1, 0])
def test_bench_prints_one_json_line(single):
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "200000", "--steps", "4",
           "--warmup", "2", "--single-pass", str(single), "--no-gather-ceiling",
           "--serve-requests", "0", "--target-iters", "0", "--no-artificial", "--no-smaller",
           "--no-cpu-baseline", "--backtrack-iters", "2"]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [l for l in out.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline", "kernels"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 4 and d["value"] > 0
    assert abs(d["value"] * d["ms_per_step"] - 1e3) < 1e-6 * 1e3
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert d["config"]["single_pass"] == bool(single) and d["config"]["n"] == 200000
    other = d["two_pass_run" if single else "single_pass_run"]
    assert other["iters_per_s"] > 0 and other["iterations"] == 4
    assert d["backtracking_run"]["trials_per_iteration"] >= 1.0
