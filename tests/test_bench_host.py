"""Host-side pieces of bench.py: the rocprofv3 counter summary that turns
FETCH_SIZE / WRITE_SIZE per dispatch into HBM bytes per launch, scaled by
what the same counters read for a copy of known size."""

import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerows(rows)


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    cal = bench.CAL_BYTES / 1024.0
    # the counters read 80% of the copy's fetched bytes and 50% of its writes
    _write(tmp_path / "cal_fetch", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 0.8 * cal),
                                    (2, "small_copy", "FETCH_SIZE", 3.0)])
    _write(tmp_path / "cal_write", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 0.5 * cal)])
    # two sparsification dispatches and an unrelated kernel; a dispatch may
    # report one counter in several rows (summed)
    _write(tmp_path / "fetch", [(7, "void k_cpqr_reg<float, 64, 3, 1>(...)", "FETCH_SIZE", 80.0),
                                (8, "void k_cpqr_coop<float, 2, true>(...)", "FETCH_SIZE", 40.0),
                                (8, "void k_cpqr_coop<float, 2, true>(...)", "FETCH_SIZE", 40.0),
                                (9, "void k_qr_reg<float, 16, 1>(...)", "FETCH_SIZE", 1e6)])
    _write(tmp_path / "write", [(7, "void k_cpqr_reg<float, 64, 3, 1>(...)", "WRITE_SIZE", 10.0),
                                (8, "void k_cpqr_coop<float, 2, true>(...)", "WRITE_SIZE", 30.0)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_2010_06807_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (tmp_path / bench.KERNEL_SOURCE).write_text("// kernels\n")
    bench.pmc_summary(str(tmp_path), "sparsify", "c4")
    out = tmp_path / bench.traffic_file("sparsify", "c4")
    t = json.loads(out.read_text())
    assert t["kernel"] == "sparsify" and t["workload"] == "c4"
    assert t["dispatches"] == [2, 2]
    assert t["scale_fetch"] == pytest.approx(1 / 0.8) and t["scale_write"] == pytest.approx(2.0)
    # per launch: fetch (80 + 80) / 2 KiB / 0.8, write (10 + 30) / 2 KiB * 2
    assert t["traffic_bytes_per_launch"] == pytest.approx(1024 * (80 / 0.8 + 20 * 2))
    # reported while the kernel source is the one measured, not after a change
    assert bench.measured_traffic("sparsify", "c4") == pytest.approx(t["traffic_bytes_per_launch"])
    assert bench.measured_traffic("sparsify", "c2") is None
    (tmp_path / bench.KERNEL_SOURCE).write_text("// kernels, changed\n")
    assert bench.measured_traffic("sparsify", "c4") is None


def test_cpu_info_and_gpus_flag(capsys, monkeypatch):
    model, avail = bench.cpu_info()
    assert isinstance(model, str) and avail >= 1
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
