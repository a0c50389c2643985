"""The benchmark's host-side contract (no GPU): one GPU only, and HBM traffic
reported only while the profiled kernel sources are the current ones."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_profiled_sources(monkeypatch):
    vals = bench.recorded_traffic()
    if vals:  # the summary matches the sources: both forms' A + W bytes are there
        chosen = "b3p" if bench.CHOSEN_OPTS.get("packed_c") else "b3"
        assert {"fp32_aw_traffic_bytes", chosen + "_aw_traffic_bytes"} <= set(vals)
        assert all(v > 0 for v in vals.values())
    monkeypatch.setattr(bench, "csrc_digest", lambda: "0" * 64)
    assert bench.recorded_traffic() == {}
