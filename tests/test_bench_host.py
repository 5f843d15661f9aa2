"""Host-side logic of bench.py that needs no GPU: the HBM-traffic record is
the march kernel's counter bytes scaled by what the same counter reads for
a plain copy of known size, and records go stale when the kernel sources
change."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(d, counter, rows):
    os.makedirs(os.path.join(d, "host"), exist_ok=True)
    with open(os.path.join(d, "host", "1_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for i, (kernel, kib) in enumerate(rows):
            w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": i + 1, "Kernel_Name": kernel,
                                                  "Counter_Name": counter, "Counter_Value": kib})


def test_traffic_record_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    calib_kib = bench.CALIB_BYTES / 1024
    fetch, write = str(tmp_path / "fetch"), str(tmp_path / "write")
    # the counter reads half of the copy's bytes: scale 2; the march reads 3 GiB by it
    _write(fetch, "FETCH_SIZE", [("ingest_kernel<float>", calib_kib / 2),
                                 ("ingest_kernel<float>", 123.0),
                                 ("march_queue<float, true>", 3 * 2 ** 20 / 2),
                                 ("march_queue<float, true>", 3 * 2 ** 20 / 2)])
    _write(write, "WRITE_SIZE", [("ingest_kernel<float>", calib_kib),
                                 ("march_queue<float, true>", 1024.0)])
    monkeypatch.setattr(bench, "traffic_path", lambda w, s: str(tmp_path / "rec.json"))
    args = type("A", (), {"summarize_pmc": [fetch, write], "workload": "c2", "storage": "f32"})
    assert bench.summarize_pmc(args) == 0
    rec = json.load(open(tmp_path / "rec.json"))
    assert rec["counters"]["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert rec["counters"]["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    assert rec["hbm_bytes_per_frame"] == pytest.approx(3 * 2 ** 30 + 1024 * 1024)
    assert bench.traffic_for("c2", "f32") == pytest.approx(rec["hbm_bytes_per_frame"])
    # a changed kernel source invalidates the record
    monkeypatch.setattr(bench, "kernel_sha256", lambda: "0" * 64)
    assert bench.traffic_for("c2", "f32") is None


def test_valu_view_uses_the_unpacked_vector_rate(tmp_path, monkeypatch):
    sq = str(tmp_path / "sq")
    insts = 2.4e9 * 256 * 1e-3            # one millisecond of wave64 VALU issue: 1 per CU per cycle
    _write(sq, "SQ_INSTS_VALU", [("march_queue<float, true>", insts)])
    monkeypatch.setattr(bench, "valu_path", lambda w, s: str(tmp_path / "valu.json"))
    args = type("A", (), {"summarize_sq": sq, "workload": "c2", "storage": "f32"})
    assert bench.summarize_sq(args) == 0
    v = bench.valu_for("c2", "f32", 2.0)
    assert v["issue_ms"] == pytest.approx(1.0)
    assert v["frac"] == pytest.approx(0.5)


def test_more_than_one_gpu_is_refused(capsys, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().out
