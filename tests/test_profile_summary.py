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
