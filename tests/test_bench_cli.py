"""Host-side checks of bench.py (no GPU): the one-GPU rule and the traffic bookkeeping."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    rec = json.load(open(bench.TRAFFIC_FILE))
    kern = "MpkBody<double, double, 1>"
    f = tmp_path / "traffic.json"
    rec["source_hash"] = bench.kernel_source_hash()
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(kern) == rec["kernels"][kern]["hbm_bytes_per_launch"]
    assert bench.measured_traffic("NoSuchBody<double>") is None
    rec["source_hash"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(kern) is None
