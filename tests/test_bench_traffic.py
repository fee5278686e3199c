"""Host logic of bench.py's traffic records (no GPU): the copy-kernel calibration of the
rocprofv3 counters, the per-kind averages over the last dispatches, the per-workload and
per-order keys, and the source-hash guard that drops a record once the kernel changed."""

import csv
import json
import os

import bench


def _write_counters(d, rows):
    """rows: (dispatch id, kernel name, KiB) -> a rocprofv3-style counter_collection.csv"""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
        w.writeheader()
        for i, name, kib in rows:
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Value": kib})


def test_summarize_traffic_scales_and_takes_the_last_dispatches(tmp_path):
    copy_bytes = 1 << 20
    # the copy kernel reads half its bytes through FETCH_SIZE and all of them through WRITE_SIZE
    _write_counters(tmp_path / "cf", [(1, "copy", copy_bytes / 2 / 1024)])
    _write_counters(tmp_path / "cw", [(1, "copy", copy_bytes / 1024)])
    k1, k2 = "void dwf::hop_kernel<1, 1, 1, false, 1, 1, false>(x)", "void dwf::hop_kernel<1, 1, 1, true, 3, 1, false>(x)"
    # two early dispatches of k1 (an autotuner's) that `last` must skip; ids out of order in the file
    fetch = [(5, k1, 10.0), (1, k1, 999.0), (2, k1, 999.0), (6, k1, 14.0), (7, k2, 20.0), (8, k2, 22.0)]
    write = [(5, k1, 4.0), (1, k1, 0.0), (2, k1, 0.0), (6, k1, 4.0), (7, k2, 8.0), (8, k2, 8.0)]
    _write_counters(tmp_path / "f", [(i, n, v / 2) for i, n, v in fetch])  # FETCH_SIZE reads half
    _write_counters(tmp_path / "w", write)
    rec = bench.summarize_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                                  str(tmp_path / "cw"), copy_bytes, prefixes=[k1[:40], k2[:40]], last=2)
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    a, b = rec["kinds"][k1[:40]], rec["kinds"][k2[:40]]
    assert a["dispatches"] == 2 and abs(a["fetch_bytes"] - 12.0 * 1024) < 1e-6 and abs(a["write_bytes"] - 4.0 * 1024) < 1e-6
    assert abs(b["fetch_bytes"] - 21.0 * 1024) < 1e-6 and abs(b["write_bytes"] - 8.0 * 1024) < 1e-6
    assert abs(rec["bytes_per_launch"] - (16.0 + 29.0) * 1024 / 2) < 1e-6


def test_traffic_records_are_keyed_by_workload_and_order_and_dropped_when_the_source_changes(tmp_path, monkeypatch):
    import hashlib

    src = tmp_path / "hop.hip"
    src.write_text("kernel v1")
    rec_file = tmp_path / "hop_traffic.json"
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    rec_file.write_text(json.dumps({
        "hop_source_sha256": digest,
        "workloads": {
            "rb_solve": {"orders": {"3:1,4,2": {"bytes_per_launch": 1.0}, "1": {"bytes_per_launch": 2.0}}},
            "batched": {"orders": {"3:1,4,2": {"bytes_per_launch": 3.0}}},
        },
    }))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec_file))
    monkeypatch.setattr(bench, "HOP_SOURCE", str(src))
    assert bench._order_key({"mode": 3, "box": [1, 4, 2]}) == "3:1,4,2" and bench._order_key({"mode": 1}) == "1"
    assert bench.measured_traffic("rb_solve", {"mode": 3, "box": [1, 4, 2]}) == 1.0
    assert bench.measured_traffic("rb_solve", {"mode": 1}) == 2.0
    assert bench.measured_traffic("batched", {"mode": 3, "box": [1, 4, 2]}) == 3.0
    assert bench.measured_traffic("batched", {"mode": 1}) is None  # no record in that order
    assert bench.measured_traffic("mixed", {"mode": 1}) is None  # no record for that workload
    src.write_text("kernel v2")  # the kernel changed since the counters were taken
    assert bench.measured_traffic("rb_solve", {"mode": 1}) is None
