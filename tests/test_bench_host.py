"""Host-side pieces of bench.py: the refusal of more than one GPU, the
algorithmic bytes per node of each step kernel, and the lookup of the committed
rocprofv3 traffic records (by workload, kernel and launch variant)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_algorithmic_bytes_per_node():
    # (2Q + 2) * 8 for the whole step; the collides move Q pulls, the force and Q + 1 writes
    assert bench.kernel_bytes_per_node("k_ring", 19, 3, "CD6") == 8 * (19 + 3 + 19 + 1) == 336
    assert bench.kernel_bytes_per_node("k_tile", 19, 3, "CD6") == 336
    assert bench.kernel_bytes_per_node("k_ring", 9, 2, "CD6") == 168
    assert bench.kernel_bytes_per_node("k_fused", 9, 2, "CD6") == 8 * (9 + 2 + 9 + 1)
    assert bench.kernel_bytes_per_node("k_mu_march", 19, 3, "CD6") == 16
    assert bench.kernel_bytes_per_node("k_force_march", 19, 3, "CD6") == 40
    assert bench.kernel_bytes_per_node("k_collide", 19, 3, "OCFDS4") == 8 * (19 + 6 + 19)
    assert bench.kernel_bytes_per_node("k_mf", 19, 3, "CD6") == 32


def test_cpu_model_is_named():
    assert bench.cpu_model() != ""


def test_traffic_record_lookup():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path))
    assert rec, "profiles/traffic.json holds no record"
    for key, ent in rec.items():
        workload, kernel = key.split(" | ")[:2]
        got = bench.traffic_record(kernel, workload, ent.get("variant"))
        if ent["source_hash"] == bench.kernel_source_hash():
            assert got == ent["bytes_per_launch"]
        else:
            assert got is None          # stale: taken on other kernel sources
        # another launch variant never borrows this record
        assert bench.traffic_record(kernel, workload, "no such variant") is None

