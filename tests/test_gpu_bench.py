"""bench.py keeps its JSON contract: one line with the metric, the run's own counts, the roofline
object for the dominant kernel and the CPU baseline object, on a small throughput lattice."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line_contract():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "512", "--steps", "40", "--warmup", "4",
           "--no-batched", "--no-warm-start"]
    print("[bench contract]", " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 40 and d["warmup"] == 4
    assert d["unit"] == "MLUPS" and d["higher_is_better"] is True and d["dtype"] == "f32"
    assert "512x512" in d["config"]["workload"]
    assert d["value"] > 0 and d["ms_per_step"] > 0
    # value is all sites per wall-clock second of the timed steps
    assert abs(d["value"] - d["config"]["n_sites"] / (d["ms_per_step"] * 1e3)) <= 1e-2 * d["value"]
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert rf["traffic"] is None  # the committed counter summary is for the 4096^2 workload
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and "512x512" in cb["sample"]
    assert "fp64" in d and d["fp64"]["value"] > 0
