"""bench.py's host-side contract: one GPU only, and the committed HBM byte
counters belong to the committed gradient + Adam kernel sources (otherwise
the bench line would report traffic as null)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_counters_match_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "k_iterate_traffic.json")) as fh:
        t = json.load(fh)
    assert t["source_sha256"] == bench.kernel_source_hash()
    b, _ = bench.counter_traffic()
    assert b == (t["fetch_kib_per_launch"] * t["fetch_scale"] +
                 t["write_kib_per_launch"] * t["write_scale"]) * 1024.0
    assert os.path.exists(os.path.join(ROOT, t["summary"]))
