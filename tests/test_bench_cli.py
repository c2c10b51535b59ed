"""bench.py on the CPU: more than one GPU is refused with a message before any GPU work, and
the measured HBM traffic is reported only for the query-kernel sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    stamp = dict(bench.KQUERY_TRAFFIC)
    monkeypatch.setattr(bench, "KQUERY_TRAFFIC", {**stamp, "sources_sha256": bench.kquery_sources_sha()})
    t = bench.kquery_traffic_bytes()
    assert t == (stamp["fetch_kib"] * stamp["fetch_scale"] + stamp["write_kib"] * stamp["write_scale"]) * 1024.0
    json.dumps({"traffic": t})
    monkeypatch.setattr(bench, "KQUERY_TRAFFIC", {**stamp, "sources_sha256": "0" * 64})
    assert bench.kquery_traffic_bytes() is None
