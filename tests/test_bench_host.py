"""Host-side pieces of bench.py: the --gpus contract and the traffic record
(reported only for the kernel sources it was measured on)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_gpus_above_one_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_matches_current_sources_or_is_dropped(monkeypatch):
    rec = bench.recorded_traffic("fp64")
    if rec is not None:
        assert rec > 0
    # any change of the hashed kernel sources invalidates the record
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", ["bench.py"])
    assert bench.recorded_traffic("fp64") is None


def test_traffic_record_missing_profile(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "absent.md"))
    assert bench.recorded_traffic("fp64") is None
