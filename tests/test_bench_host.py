"""Host-side logic of bench.py (no GPU): the HBM traffic record is used only when it was
taken on the current library sources and the same workload, and more than one GPU is
refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.fixture
def traffic_dir(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"source_sha256": "abc",
           "kernels": {"k": {"workload": "w", "launches": 2, "bytes_per_launch": 10.0}}}
    with open(tmp_path / "profiles" / "traffic.json", "w") as fh:
        json.dump(rec, fh)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "abc")
    return tmp_path


def test_traffic_record_used_for_matching_sources_and_workload(traffic_dir):
    assert bench.recorded_traffic("k", "w") == 10.0
    assert bench.recorded_traffic_entry("k", "w")["launches"] == 2


def test_traffic_record_ignored_for_other_workload_or_kernel(traffic_dir):
    assert bench.recorded_traffic("k", "another workload") is None
    assert bench.recorded_traffic("other kernel", "w") is None


def test_traffic_record_ignored_once_sources_change(traffic_dir, monkeypatch):
    monkeypatch.setattr(bench, "source_hash", lambda: "changed")
    assert bench.recorded_traffic("k", "w") is None


def test_source_hash_covers_library_sources():
    h = bench.source_hash()
    assert len(h) == 64 and int(h, 16) >= 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert "one GPU" in (r.stdout + r.stderr)
