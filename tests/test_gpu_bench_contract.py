"""bench.py's output contract on a small grid: one JSON line with the metric,
the throughput and the step accounting, the roofline of the dominant kernel
(with the measured ceiling of the access pattern), and the CPU baseline of the
oracle.  Runs bench.py as a child process, as it is run on its own."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # --no-learned: the learned-start comparison runs on the batched kernel's
    # cooperative launches, which the runtime refuses in a second process
    # while this one holds the device (test_gpu_learned_gain runs it here)
    out = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--n", "64", "--steps", "5",
                          "--warmup", "2", "--cpu-steps", "1", "--no-learned"], capture_output=True, text=True,
                         timeout=240, cwd=ROOT)
    print(out.stderr[-2000:], flush=True)
    assert out.returncode == 0
    lines = [l for l in out.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "timed_step_range"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 2 and d["dtype"] == "f64"
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["config"]["workload"].startswith("D3Q19 64^3")
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert 0 < r["frac"] < 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert "traffic" in r and r["kernel"] in r["phases_ms"]
    c = r["ceiling"]
    assert c["pull_copy_GBps"] > 0 and c["aligned_copy_GBps"] > 0
    b = d["cpu_baseline"]
    assert b["kind"] == "oracle" and b["value"] > 0 and b["cores"] >= 1 and b["unit"] == "MLUPS" and b["sample"]
    first, last = d["timed_step_range"]
    assert last - first + 1 == 5
