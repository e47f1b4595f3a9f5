"""bench.py's output contract: one JSON line with the metric, the whole-job
value, the timing fields and the roofline of the dominant kernel, and a
refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_bench_prints_one_json_line_with_the_contract_fields():
    print("CASE bench contract, 5 steps", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "2", "--no-cpu-baseline",
           "--no-extras", "--no-copy-ceiling"]
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, lines
    b = json.loads(lines[0])
    assert b["unit"] == "MLUPS" and b["n_gpus"] == 1 and b["steps"] == 5 and b["warmup"] == 2
    assert b["higher_is_better"] is True and b["scaling"] == "weak" and b["data"] == "synthetic"
    assert isinstance(b["metric"], str) and isinstance(b["dtype"], str)
    assert isinstance(b["config"]["workload"], str)
    # value is the whole job's throughput over the timed steps: 256^3 cells per step
    assert b["value"] > 0 and b["ms_per_step"] > 0
    assert abs(b["value"] - 256 ** 3 / (b["ms_per_step"] * 1e-3) / 1e6) <= 0.01 * b["value"]
    roof = b["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert 0 < roof["achieved"] <= roof["peak"]
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert roof["traffic"] is None or roof["traffic"] > 0
    # the counter-based figures are null when the committed profile was taken
    # on another kernel source or tile height
    rv = b["roofline_valu"]
    assert rv is None or (rv["bound"] == "alu" and rv["unit"] == "G wave-instructions/s" and 0 < rv["frac"] <= 1)
    assert b["fp32"]["value"] > 0 and b["fp32"]["roofline"]["frac"] > 0
