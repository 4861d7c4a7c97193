"""bench.py's host-side contract (no GPU): one GPU only, and measured HBM traffic is reported only
for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus_requested"] == 2


def test_traffic_record_applies_only_to_matching_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps({
        "cfg2:2000:256": {"source_hash": h, "hbm_bytes_per_launch": 123.0},
        "cfg3:1000:1024": {"source_hash": "0" * 16, "hbm_bytes_per_launch": 456.0}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("cfg2:2000:256") == 123.0
    assert bench.measured_traffic("cfg3:1000:1024") is None     # kernels changed since
    assert bench.measured_traffic("cfg1:1000:16") is None       # never measured
