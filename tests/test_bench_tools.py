"""The measurement tools of bench.py that run without a GPU: the HBM-traffic derivation
from rocprofv3 counter files and the kernel-trace summary (CPU, synthetic inputs)."""
import csv
import os
import sqlite3
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KM = "void rr::k_ksym_mma<1, 16, 1, double>(long, float const*, float const*, float, double const*)"


def _counter_csv(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_from_counters_scales_by_the_copy(tmp_path):
    # the copy reads 1 GiB: FETCH_SIZE counts it as half (2x scale), WRITE_SIZE in full
    _counter_csv(str(tmp_path / "FETCH_SIZE" / "FETCH_SIZE_counter_collection.csv"), "FETCH_SIZE",
                 [("__amd_rocclr_copyBuffer", 524288.0), ("__amd_rocclr_copyBuffer", 1.5),
                  (KM, 100.0), (KM, 300.0), (KM, 200.0), ("rr::k_other", 9e9)])
    _counter_csv(str(tmp_path / "WRITE_SIZE" / "WRITE_SIZE_counter_collection.csv"), "WRITE_SIZE",
                 [("__amd_rocclr_copyBuffer", 1048576.0), (KM, 50.0), (KM, 70.0), (KM, 60.0)])
    out = tmp_path / "traffic.json"
    t = bench.traffic_from_counters(str(tmp_path), str(out))["k_ksym_mma"]
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    # medians 200 KiB fetched and 60 KiB written, scaled
    assert t["fetch_bytes"] == pytest.approx(2.0 * 200 * 1024)
    assert t["write_bytes"] == pytest.approx(60 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(t["fetch_bytes"] + t["write_bytes"])
    assert t["src_hash"] == bench._src_hash(*bench.TRAFFIC_SOURCES)
    assert out.exists()
    # the bench reads it back only under the same source hash
    assert bench._src_hash(*bench.TRAFFIC_SOURCES) == t["src_hash"]


def test_traffic_from_counters_needs_the_calibration_copy(tmp_path):
    _counter_csv(str(tmp_path / "FETCH_SIZE" / "FETCH_SIZE_counter_collection.csv"), "FETCH_SIZE", [(KM, 1.0)])
    _counter_csv(str(tmp_path / "WRITE_SIZE" / "WRITE_SIZE_counter_collection.csv"), "WRITE_SIZE", [(KM, 1.0)])
    with pytest.raises(SystemExit):
        bench.traffic_from_counters(str(tmp_path))


def test_trace_summary_table(tmp_path):
    db = str(tmp_path / "t.db")
    c = sqlite3.connect(db)
    c.execute("create table rocpd_info_kernel_symbol (id integer, guid text, display_name text)")
    c.execute("create table rocpd_kernel_dispatch (kernel_id integer, guid text, start integer, end integer)")
    c.executemany("insert into rocpd_info_kernel_symbol values (?, 'g', ?)", [(1, "k_big"), (2, "k_small")])
    # k_big: 3 working launches of 100 us and one no-op of 2 us; k_small: 2 launches of 10 us
    disp = [(1, 0, 100_000), (1, 0, 100_000), (1, 0, 100_000), (1, 0, 2_000), (2, 0, 10_000), (2, 0, 10_000)]
    c.executemany("insert into rocpd_kernel_dispatch values (?, 'g', ?, ?)", disp)
    c.commit()
    c.close()
    out = bench.trace_summary(db, top=5).splitlines()
    assert out[0] == "Total kernel time 0.3 ms over 6 launches."
    big = [l for l in out if "`k_big`" in l][0].split("|")
    # calls, total ms, avg us, avg us (work), work calls
    assert big[2].strip() == "4" and big[3].strip() == "0.30"
    assert big[4].strip() == "75.50" and big[5].strip() == "100.00" and big[6].strip() == "3"
    # sorted by total time: k_big first
    assert out.index([l for l in out if "`k_big`" in l][0]) < out.index([l for l in out if "`k_small`" in l][0])
