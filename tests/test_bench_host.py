"""Host-side logic of bench.py (no GPU): the roofline arithmetic, the HBM
counter parsing and its calibration, the stale-counter check, and the refusal
of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr
    assert res.stdout == ""  # no JSON line


def _agg(sieve_ms, part_ms, join_ms, n_part, n_join, steps=1):
    return {"kernel_ms": {"sieve": sieve_ms, "partition": part_ms, "join": join_ms, "verify": 0.1, "radicals": 0.0},
            "launches": {"sieve": steps, "partition": n_part, "join": n_join, "verify": steps, "radicals": 0}}


def test_roofline_numbers_follow_their_definitions():
    # Two steps of a search over 2^36 integers keeping 7.3e9 entries; 128
    # partition and 128 join launches per step.
    N, E, steps = 1 << 36, 7_338_536_668, 2
    agg = _agg(2 * 164.0, 2 * 45.0, 2 * 25.0, 256, 256, steps)
    dominant, roof = bench.roofline_from(agg, N, E, steps, {})
    assert dominant == "sieve"
    s = roof["sieve"]
    # 21 ops per integer over one launch of 164 ms, against 256 CU x 64 x 2.4 GHz.
    assert s["avg_launch_ms"] == pytest.approx(164.0)
    assert s["achieved"] == pytest.approx(21.0 * N / 0.164 / 1e12)
    assert s["peak"] == pytest.approx(39.3216)
    assert s["frac"] == pytest.approx(s["achieved"] / s["peak"])
    assert s["traffic"] is None
    # Partition: a 12 B read and a 12 B write per entry; 128 launches per step.
    p = roof["partition"]
    assert p["bytes_per_launch"] == pytest.approx(24 * E / 128)
    assert p["achieved"] == pytest.approx(24 * E / 128 / (45.0 / 128 * 1e-3) / 1e9)
    assert p["frac"] == pytest.approx(p["achieved"] / 8000.0)
    # Join: one 12 B read per entry.
    j = roof["join"]
    assert j["bytes_per_launch"] == pytest.approx(12 * E / 128)
    assert j["frac"] == pytest.approx(12 * E / 0.025 / 1e9 / 8000.0)
    # The join side as a whole: 24 B per kept key over both kernels' time.
    assert roof["join_total"]["achieved"] == pytest.approx(24 * E / 0.070 / 1e9)
    # A workload where the join kernels dominate names them.
    dominant, _ = bench.roofline_from(_agg(1.0, 5.0, 9.0, 4, 4), N, E, 1, {})
    assert dominant == "join"


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_counter_parsing_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    kib = bench.CALIB_BYTES / 1024
    copy = "void at::native::elementwise_kernel<copy_kernel>(...)"
    # FETCH_SIZE reads half the copy's known bytes (scale 2), WRITE_SIZE all of them (scale 1).
    _write_counters(tmp_path / "f", "FETCH_SIZE", [
        (copy, kib / 2),
        ("void bx::k_sieve<8192, 1024, 1>(bx::SieveParams)", 1000.0),
        ("void bx::k_partition<1024, false>(bx::PartParams)", 10.0),
        ("void bx::k_partition<1024, false>(bx::PartParams)", 30.0),
        ("void bx::k_join<1024>(bx::JoinParams)", 7.0),
        ("void bx::k_join_sort<1024>(bx::JoinParams)", 999999.0),  # another kernel: not the join
    ])
    _write_counters(tmp_path / "w", "WRITE_SIZE", [
        (copy, kib),
        ("void bx::k_sieve<8192, 1024, 1>(bx::SieveParams)", 2000.0),
        ("void bx::k_partition<1024, false>(bx::PartParams)", 20.0),
        ("void bx::k_partition<1024, false>(bx::PartParams)", 40.0),
        ("void bx::k_join<1024>(bx::JoinParams)", 0.5),
    ])
    bench.parse_counters(str(tmp_path / "f"), str(tmp_path / "w"))
    t = json.load(open(out))
    assert t["fetch_scale"] == pytest.approx(2.0)
    assert t["write_scale"] == pytest.approx(1.0)
    k = t["kernels"]
    assert k["sieve"]["fetch_bytes_per_launch"] == pytest.approx(1000.0 * 1024 * 2)
    assert k["sieve"]["write_bytes_per_launch"] == pytest.approx(2000.0 * 1024)
    # Per-launch averages over the launches of a kernel.
    assert k["partition"]["launches"] == 2
    assert k["partition"]["fetch_bytes_per_launch"] == pytest.approx(20.0 * 1024 * 2)
    assert k["partition"]["write_bytes_per_launch"] == pytest.approx(30.0 * 1024)
    assert k["join"]["launches"] == 1
    assert k["join"]["fetch_bytes_per_launch"] == pytest.approx(7.0 * 1024 * 2)
    # The file is tagged with the current kernel sources and is read back as bytes per launch.
    assert t["source_hash"] == bench.kernel_source_hash()
    traffic = bench.load_traffic()
    assert traffic["join"][0] == pytest.approx(7.0 * 1024 * 2 + 0.5 * 1024) and traffic["join"][1] == 1
    # Reported only for a run with as many launches per search as the counters saw.
    assert bench.traffic_of(traffic, "partition", 6, 3) == pytest.approx(20.0 * 1024 * 2 + 30.0 * 1024)
    assert bench.traffic_of(traffic, "partition", 4, 3) is None
    assert bench.traffic_of(traffic, "verify", 1, 1) is None


def test_stale_counters_are_not_reported(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    json.dump({"source_hash": "0" * 16, "kernels": {"join": {"fetch_bytes_per_launch": 1.0,
                                                             "write_bytes_per_launch": 1.0}}}, open(out, "w"))
    assert bench.load_traffic() == {}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.load_traffic() == {}



def test_cpu_baseline_reports_its_sample_cores_and_cpu():
    cb = bench.cpu_baseline(1 << 20, 12)  # 4097 integers: milliseconds
    assert cb["kind"] == "oracle" and cb["unit"] == "integers/s"
    assert 1 <= cb["cores"] <= 16
    assert cb["value"] > 0 and cb["seconds"] > 0
    assert "[1044480, 1048577)" in cb["sample"]
    assert "cpu_model" in cb


def test_trace_overlap_counts_time_with_two_streams_running(tmp_path):
    # Stream A runs [0, 100) and [300, 400) ns; stream B runs [50, 150) and [160, 170) ns
    # (two kernels of one stream that touch do not count as overlap).
    rows = [(0, 100, 1), (300, 400, 1), (50, 150, 2), (160, 170, 2), (170, 180, 2)]
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Queue_Id", "Stream_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for t0, t1, st in rows:
            w.writerow({"Queue_Id": st, "Stream_Id": st, "Kernel_Name": "k", "Start_Timestamp": t0,
                        "End_Timestamp": t1})
    out = bench.trace_overlap(str(tmp_path))
    assert out["kernels"] == 5
    assert len(out["streams"]) == 2
    # Busy: [0, 150) + [160, 180) + [300, 400) = 270 ns; two streams at once: [50, 100) = 50 ns.
    assert out["busy_ms"] == pytest.approx(270e-6)
    assert out["overlap_ms"] == pytest.approx(50e-6)
    assert out["overlap_frac_of_busy"] == pytest.approx(50 / 270)
