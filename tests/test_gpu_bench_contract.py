"""bench.py's output line, on a small grid: one JSON line on stdout with the
fields its readers depend on, a roofline object priced against the
published FP64 peak, and no HBM traffic figure for a grid the counter runs
did not cover."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_on_a_small_grid():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "256", "--steps", "4", "--warmup", "2",
           "--no-cpu-baseline", "--no-extra"]
    print("[bench contract]", " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 4 and d["warmup"] == 2
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert abs(d["value"] - 256 * 256 / (d["ms_per_step"] * 1e-3)) <= 1e-9 * d["value"]
    assert d["higher_is_better"] is True and d["dtype"] == "f64" and d["vs_baseline"] is None
    assert d["metric"].endswith("256^2") and "256x256" in d["config"]["workload"]
    rf = d["roofline"]
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    assert 0 < rf["frac"] < 1 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-12
    assert rf["traffic"] is None          # the counters cover 2048^2, steps 5-24 only
    assert d["device_status"] == 0
    assert d["graph_replayed"]["same_final_state_as_eager"] is True
