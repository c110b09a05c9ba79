"""The rocprofv3 summaries (no GPU): synthetic counter files with known answers."""
from __future__ import annotations

import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(("Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"), r)))


def _run(*args):
    return subprocess.run([sys.executable, "-m", "paper_1807_03749_amd.profile_summary", *args], cwd=ROOT,
                          capture_output=True, text=True, check=True).stdout


def test_traffic_scales_by_the_copy_calibration(tmp_path):
    # kernel: 100 KiB fetched, 50 KiB written per dispatch (two dispatches, one split over two
    # counter instances); copies of 1 MiB x 5 read back half their bytes and all of them
    k = "void ccmc::k_items<2, double>(args)"
    _counters(tmp_path / "f.csv", [(1, k, "FETCH_SIZE", 100), (2, k, "FETCH_SIZE", 60), (2, k, "FETCH_SIZE", 40)])
    _counters(tmp_path / "w.csv", [(1, k, "WRITE_SIZE", 50), (2, k, "WRITE_SIZE", 50)])
    _counters(tmp_path / "cf.csv", [(9, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 2560.0)])
    _counters(tmp_path / "cw.csv", [(9, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 5120.0)])
    out = _run("traffic", "--kernel", "k_items<", "--name", "items", "--workload", "w", "--fetch", str(tmp_path / "f.csv"),
               "--write", str(tmp_path / "w.csv"), "--copy-fetch", str(tmp_path / "cf.csv"), "--copy-write",
               str(tmp_path / "cw.csv"), "--copy-bytes", str(1 << 20), "--command", "test")
    got = dict(ln.split(" = ", 1) for ln in out.splitlines() if " = " in ln and not ln.startswith("#"))
    assert got["dispatches_fetch"] == "2" and float(got["fetch_kib_per_dispatch"]) == 100.0
    assert float(got["hbm_bytes_per_launch"]) == (100 * 2.0 + 50 * 1.0) * 1024


def test_valu_busy_divides_the_xcd_sum(tmp_path):
    # 1024 SIMDs busy half the time for 1000 cycles: 4 * ACTIVE / (1024 * 8000 / 8) = 0.5
    k = "void ccmc::k_generate<2, double>(args)"
    _counters(tmp_path / "v.csv", [(1, k, "SQ_WAVES", 100), (1, k, "SQ_INSTS_VALU", 5000),
                                   (1, k, "SQ_ACTIVE_INST_VALU", 128000), (1, k, "SQ_WAVE_CYCLES", 1000),
                                   (1, k, "SQ_WAIT_INST_ANY", 250), (1, k, "GRBM_GUI_ACTIVE", 8000)])
    out = _run("valu", "--pmc", str(tmp_path / "v.csv"), "--kernels", "k_generate<", "--workload", "w", "--command", "t")
    row = [ln for ln in out.splitlines() if ln.strip().startswith("k_generate<")][0].split()
    assert row[1] == "1" and float(row[3]) == 50.0 and row[4] == "50.0%" and row[5] == "25.0%"


def test_gaps_sum_the_idle_time_between_kernels(tmp_path):
    # two steps of three kernels; in the last step the GPU waits 4 us before k_items and 1 us
    # before k_final_part; hipLaunchKernel takes 7 us per call
    seq = [("k_guide", 0, 10), ("k_items", 10, 20), ("k_final_part", 20, 25),
           ("k_guide", 30, 40), ("k_items", 44, 60), ("k_final_part", 61, 65)]
    with open(tmp_path / "k.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i, (n, s, e) in enumerate(seq):
            w.writerow({"Kernel_Name": f"void ccmc::{n}(args)", "Correlation_Id": i, "Start_Timestamp": s * 1000,
                        "End_Timestamp": e * 1000})
    with open(tmp_path / "a.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Function", "Correlation_Id", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i in range(len(seq)):
            w.writerow({"Function": "hipLaunchKernel", "Correlation_Id": i, "Start_Timestamp": 0, "End_Timestamp": 7000})
    out = _run("gaps", str(tmp_path / "k.csv"), "--steps", "1", "--api", str(tmp_path / "a.csv"), "--command", "t")
    rows = {tuple(ln.split()[:3:2]): float(ln.split()[-1]) for ln in out.splitlines() if "->" in ln and not ln.startswith("#")}
    assert rows[("k_guide", "k_items")] == 4.0 and rows[("k_items", "k_final_part")] == 1.0
    assert "per step: 5.0 us idle" in out and "median 7.00 us" in out
