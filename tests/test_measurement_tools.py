"""Host logic of the measurement tools (no GPU): the counter summary's
calibration arithmetic and the benchmark's rule for reporting HBM traffic
only under the kernel source and schedule the counters ran with."""
import csv
import hashlib
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_pmc_summary_calibration(tmp_path):
    from paper_1405_4644_amd import pmc_summary
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    # two dispatches of the kernel (the second split over two counter rows, as
    # per-XCD instances are), one of another kernel that must be ignored
    _csv(tmp_path / "f.csv", [
        {"Dispatch_Id": 1, "Kernel_Name": "void k_up<128>(float*)", "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000},
        {"Dispatch_Id": 2, "Kernel_Name": "void k_up<128>(float*)", "Counter_Name": "FETCH_SIZE", "Counter_Value": 1500},
        {"Dispatch_Id": 2, "Kernel_Name": "void k_up<128>(float*)", "Counter_Name": "FETCH_SIZE", "Counter_Value": 500},
        {"Dispatch_Id": 3, "Kernel_Name": "void k_up<64>(float*)", "Counter_Name": "FETCH_SIZE", "Counter_Value": 9e9}])
    _csv(tmp_path / "w.csv", [
        {"Dispatch_Id": 1, "Kernel_Name": "void k_up<128>(float*)", "Counter_Name": "WRITE_SIZE", "Counter_Value": 300},
        {"Dispatch_Id": 2, "Kernel_Name": "void k_up<128>(float*)", "Counter_Name": "WRITE_SIZE", "Counter_Value": 500}])
    # the copy of 1 MiB: FETCH_SIZE reads half the bytes, WRITE_SIZE all of them
    _csv(tmp_path / "cf.csv", [
        {"Dispatch_Id": 1, "Kernel_Name": "fill", "Counter_Name": "FETCH_SIZE", "Counter_Value": 3},
        {"Dispatch_Id": 2, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": 512}])
    _csv(tmp_path / "cw.csv", [
        {"Dispatch_Id": 2, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "WRITE_SIZE", "Counter_Value": 1024}])
    out = tmp_path / "rec.json"
    pmc_summary.main(["--fetch", str(tmp_path / "f.csv"), "--write", str(tmp_path / "w.csv"),
                      "--cal-fetch", str(tmp_path / "cf.csv"), "--cal-write", str(tmp_path / "cw.csv"),
                      "--cal-bytes", str(1 << 20), "--kernel-regex", r"k_up<128>", "--source", str(src),
                      "--schedule", "6,448,0", "--out", str(out)])
    rec = json.loads(out.read_text())
    assert rec["dispatches"] == 2
    assert rec["fetch_kib_per_dispatch"] == pytest.approx(1500.0)  # (1000 + 2000) / 2
    assert rec["copy_calibration"]["fetch_factor"] == pytest.approx(0.5)
    assert rec["copy_calibration"]["write_factor"] == pytest.approx(1.0)
    assert rec["hbm_read_bytes_per_launch"] == pytest.approx(1500.0 * 1024 / 0.5)
    assert rec["hbm_write_bytes_per_launch"] == pytest.approx(400.0 * 1024)
    assert rec["schedule"] == {"group": 6, "upd_slots": 448, "small_tiles": 0}
    assert rec["source_sha256"] == hashlib.sha256(b"kernel source").hexdigest()


def test_traffic_reported_only_under_the_recorded_schedule():
    import bench
    with open(os.path.join(ROOT, "profiles", "pmc_k_syrk_update_fp32_n16384.json")) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_1405_4644_amd", "csrc", "k_update.hip"), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == rec["source_sha256"]
    got = bench.measured_traffic("fp32", dict(rec["schedule"]))
    assert (got is not None) == current
    other = dict(rec["schedule"], group=rec["schedule"]["group"] + 1)
    assert bench.measured_traffic("fp32", other) is None
    assert bench.measured_traffic("fp64", dict(rec["schedule"])) is None  # no record for binary64
