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


def test_traffic_counters_only_for_their_kernel_and_workload(tmp_path, monkeypatch):
    # the committed HBM byte counters are used only while the kernel sources
    # hash to the value they were taken on and for the workload they were
    # taken on; otherwise traffic is null
    sys.path.insert(0, ROOT)
    import bench
    t = {"kernel": "k_iterate", "workload": "w", "source_sha256": bench.kernel_source_hash(),
         "fetch_kib_per_launch": 100.0, "write_kib_per_launch": 50.0, "fetch_scale": 2.0,
         "write_scale": 1.0, "summary": "profiles/x.md"}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    b, _ = bench.counter_traffic("w")
    assert b == (100.0 * 2.0 + 50.0 * 1.0) * 1024.0
    assert bench.counter_traffic("other")[0] is None
    t["source_sha256"] = "0" * 64
    f.write_text(json.dumps(t))
    assert bench.counter_traffic("w")[0] is None


def test_committed_counter_summary_exists():
    with open(os.path.join(ROOT, "profiles", "k_iterate_traffic.json")) as fh:
        t = json.load(fh)
    assert os.path.exists(os.path.join(ROOT, t["summary"]))
    for k in ("workload", "source_sha256", "fetch_kib_per_launch", "write_kib_per_launch",
              "fetch_scale", "write_scale", "commands"):
        assert k in t, k


def test_committed_counters_match_the_committed_kernel():
    # the counters were taken on the kernel sources as committed, so the
    # bench line carries traffic; and the summary they point to names the
    # same source hash.  Traffic lies near the algorithmic bytes of the
    # C3 state (176 N + 4 (N + nnz), N = 1e6, nnz / N = 2.305): above it by
    # the whole-record writes, below 1.5 x (no gross re-reads)
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    assert t["source_sha256"] == bench.kernel_source_hash()
    with open(os.path.join(ROOT, t["summary"])) as fh:
        assert t["source_sha256"] in fh.read()
    b, _ = bench.counter_traffic(t["workload"])
    algorithmic = 176.0 * 1e6 + 4.0 * (1e6 + 2.305e6)
    assert 0.9 * algorithmic < b < 1.5 * algorithmic
