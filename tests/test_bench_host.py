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


def test_counter_summary_groups_by_kernel_name_from_the_round_trip(tmp_path, capsys):
    """Shader counters are summed per bench kernel name over the dispatches from two before the
    first forward-SHT table product on; earlier dispatches (plan creation) are left out."""
    rows = [("0", "void s2w::k_lsum_bf3_list<4>(x)", 99.0),   # before the window: ignored
            ("3", "s2w::k_sht_tab(s2w::ShtTab)", 1.0),
            ("4", "void s2w::k_lsum_bf3_list<4>(x)", 1.0),
            ("5", "void s2w::k_lsum_bf3<2, 4>(x)", 1.0)]
    counters = {"SQ_WAVE_CYCLES": 100.0, "SQ_BUSY_CYCLES": 10.0, "SQ_WAIT_INST_ANY": 25.0,
                "SQ_VALU_MFMA_BUSY_CYCLES": 64.0, "SQ_INSTS_MFMA": 4.0, "SQ_INSTS_VALU": 40.0,
                "SQ_INSTS_LDS": 8.0, "SQ_LDS_BANK_CONFLICT": 4.0}
    with open(tmp_path / "run_counter_collection.csv", "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, k, scale in rows:
            for c, v in counters.items():
                fh.write(f'{d},"{k}",{c},{v * scale}\n')
    bench.summarize_counters(str(tmp_path))
    out = capsys.readouterr().out
    lsum = [ln for ln in out.splitlines() if ln.startswith("| lsum_mm |")]
    # two dispatches in the window; busy = 128 / (20 x 32), waiting 50 / 200, 80 / 8 VALU per MFMA
    assert lsum == ["| lsum_mm | 2 | 0.200 | 0.250 | 10.0 | 0.50 |"]
    assert any(ln.startswith("| sht_tab | 1 |") for ln in out.splitlines())
