"""Host-side helpers of bench.py that turn rocprofv3 output into the numbers
the bench line reports (no GPU: the CSV files are written here)."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_counter_per_dispatch_sums_rows_of_a_dispatch(tmp_path):
    rows = []
    for d, vals in ((1, (10, 20)), (2, (30, 40))):
        for v in vals:   # two rows per dispatch (e.g. one per shader engine)
            rows.append({"Dispatch_Id": d, "Kernel_Name": "void omap::k_sweep_split<16>(omap::RoundArgs)",
                         "Counter_Name": "SQ_INSTS_LDS", "Counter_Value": v})
    rows.append({"Dispatch_Id": 3, "Kernel_Name": "omap::k_walk(int)", "Counter_Name": "SQ_INSTS_LDS",
                 "Counter_Value": 1000})
    _write_csv(str(tmp_path / "a" / "1_counter_collection.csv"), rows)
    mean, n = bench._counter_per_dispatch(str(tmp_path), "SQ_INSTS_LDS", "omap::k_sweep_split<")
    assert n == 2 and mean == pytest.approx(50.0)
    with pytest.raises(SystemExit):
        bench._counter_per_dispatch(str(tmp_path), "SQ_WAVES", "omap::k_sweep_split<")


def test_kernel_avg_us_weights_by_calls(tmp_path):
    _write_csv(str(tmp_path / "b" / "1_kernel_stats.csv"), [
        {"Name": "omap::k_walk(int)", "Calls": 3, "TotalDurationNs": 3000},
        {"Name": "omap::k_walk(int)", "Calls": 1, "TotalDurationNs": 5000},
        {"Name": "omap::k_fill(int)", "Calls": 9, "TotalDurationNs": 9},
    ])
    assert bench._kernel_avg_us(str(tmp_path), "omap::k_walk(") == pytest.approx(2.0)


def test_committed_summaries_match_their_sources():
    """A committed counter summary is used by the bench line only while the
    kernel sources it was taken on are unchanged (its hash)."""
    for path, files in ((bench.TRAFFIC_FILE, bench.KERNEL_SOURCES), (bench.LDS_FILE, bench.LDS_SOURCES)):
        if not os.path.exists(path):
            continue
        with open(path) as f:
            t = json.load(f)
        assert t["kernel_sources"] == list(files)
        assert len(t["kernel_source_sha256"]) == 64


def test_more_than_one_gpu_is_refused():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_summaries_of_other_sources_are_not_reported(tmp_path, monkeypatch):
    """measured_traffic / measured_lds give None when the summary's source hash,
    workload or options differ from the run's."""
    t = {"kernel_source_sha256": "0" * 64, "workload": "w", "options": {"a": 1}, "bytes_per_launch": 5,
         "kernels": {"k": {}}}
    for attr, fn in (("TRAFFIC_FILE", bench.measured_traffic), ("LDS_FILE", bench.measured_lds)):
        path = tmp_path / (attr + ".json")
        path.write_text(json.dumps(t))
        monkeypatch.setattr(bench, attr, str(path))
        assert fn("w", {"a": 1}) is None            # other sources
        good = dict(t, kernel_source_sha256=bench.kernel_source_hash(
            bench.KERNEL_SOURCES if attr == "TRAFFIC_FILE" else bench.LDS_SOURCES))
        path.write_text(json.dumps(good))
        assert fn("w", {"a": 1}) is not None
        assert fn("other", {"a": 1}) is None
        assert fn("w", {"a": 2}) is None
