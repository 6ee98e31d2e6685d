"""Host logic of the profiling summaries (CPU only): the kernel table, the
per-dispatch counter medians, and the calibrated HBM traffic that the
benchmark reads for its roofline, on small synthetic rocprofv3 CSV files."""

from __future__ import annotations

import csv
import json

import pytest

from paper_2204_11762_amd import rocprof_summary as rs

SHA = "ab" * 32
BF16 = "void mfa::(anonymous namespace)::render_brick_kernel<3, 1, true, true, true, 4, false>(mfa::RenderArgsDev)"
BF16_VALUE = "void mfa::(anonymous namespace)::render_brick_kernel<3, 1, false, true, true, 4, false>(mfa::RenderArgsDev)"
FP32 = "void mfa::(anonymous namespace)::render_brick_kernel<3, 0, true, true, true, 4, false>(mfa::RenderArgsDev)"
COPY = "__amd_rocclr_copyBuffer"


def _write_counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter,
                        "Counter_Value": value})


def test_kernel_table_sorted_by_total_and_names_shortened(tmp_path):
    stats = tmp_path / "run_kernel_stats.csv"
    with open(stats, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs",
                                           "MinNs", "MaxNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "mfa::(anonymous namespace)::plan_cost_kernel(int*)", "Calls": 4,
                    "TotalDurationNs": 32000, "AverageNs": 8000, "MinNs": 7000,
                    "MaxNs": 9000, "Percentage": 1.0})
        w.writerow({"Name": BF16, "Calls": 4, "TotalDurationNs": 2.6e6, "AverageNs": 6.5e5,
                    "MinNs": 6.0e5, "MaxNs": 7.0e5, "Percentage": 99.0})
    rows = rs.kernel_table(str(stats))
    assert [r["calls"] for r in rows] == [4, 4]
    assert rs.short_name(rows[0]["name"]) == "render_brick_kernel<3, 1, true, true, true, 4, false>"
    assert rs.short_name(rows[1]["name"]) == "plan_cost_kernel"
    log = tmp_path / "bench.log"
    log.write_text(f"[bench] kernel source sha256 {SHA}\n[bench] store=bf16: x\nnoise\n"
                   "[bench] batch: 64 requests\n[bench] serve: 800 requests\n"
                   "[bench] eval fp32 random: 1 ms\n")
    out = tmp_path / "k.txt"
    rs.main(["kernels", str(stats), "--title", "t", "--command", "cmd", "--out", str(out),
             "--bench-log", str(log)])
    text = out.read_text()
    assert "# command: cmd" in text and "650.00" in text
    assert "[bench] store=bf16: x" in text and "[bench] batch: 64 requests" in text
    assert "[bench] serve: 800 requests" in text
    assert "noise" not in text and "eval fp32 random" not in text


def test_counters_median_per_unit_and_per_lane(tmp_path):
    a = tmp_path / "a.csv"
    _write_counters(a, [(BF16, "SQ_INSTS_VALU", 100.0), (BF16, "SQ_INSTS_VALU", 300.0),
                        (BF16, "SQ_INSTS_VALU", 200.0), (FP32, "SQ_INSTS_VALU", 9e9),
                        (BF16, "GRBM_GUI_ACTIVE", 50.0)])
    out = tmp_path / "c.txt"
    rs.main(["counters", str(a), "--kernel", "render_brick_kernel<3, 1, true", "--per", "64",
             "--unit", "sample", "--title", "t", "--command", "c1", "--out", str(out)])
    lines = {ln.split()[0]: ln.split() for ln in out.read_text().splitlines()
             if ln.startswith(("SQ_", "GRBM_"))}
    # median of the matching dispatches only; per unit; x64 per unit for SQ_INSTS_*
    assert lines["SQ_INSTS_VALU"][1:3] == ["3", "200"]
    assert float(lines["SQ_INSTS_VALU"][5]) == pytest.approx(200.0 / 64)
    assert float(lines["SQ_INSTS_VALU"][6]) == pytest.approx(200.0)
    assert len(lines["GRBM_GUI_ACTIVE"]) == 6


def test_traffic_scaled_by_the_calibration_copy(tmp_path):
    mib = 256
    copy_bytes = mib << 20
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # FETCH_SIZE reads half the copied bytes (2 bytes per counted byte),
    # WRITE_SIZE reads them exactly; a smaller copy of the run is ignored
    _write_counters(fetch, [(COPY, "FETCH_SIZE", copy_bytes / 2 / 1024),
                            (COPY, "FETCH_SIZE", 10.0),
                            (BF16, "FETCH_SIZE", 1000.0), (BF16, "FETCH_SIZE", 1200.0),
                            (BF16, "FETCH_SIZE", 1100.0), (BF16_VALUE, "FETCH_SIZE", 900.0),
                            (FP32, "FETCH_SIZE", 2000.0)])
    _write_counters(write, [(COPY, "WRITE_SIZE", copy_bytes / 1024),
                            (BF16, "WRITE_SIZE", 300.0), (BF16_VALUE, "WRITE_SIZE", 310.0),
                            (FP32, "WRITE_SIZE", 320.0)])
    flog, wlog = tmp_path / "f.log", tmp_path / "w.log"
    for p in (flog, wlog):
        p.write_text(f"[bench] kernel source sha256 {SHA}\n")
    out = tmp_path / "t.json"
    rs.main(["traffic", "--fetch", str(fetch), "--write", str(write), "--fetch-log", str(flog),
             "--write-log", str(wlog), "--fetch-command", "cf", "--write-command", "cw",
             "--copy-mib", str(mib), "--out", str(out)])
    rec = json.loads(out.read_text())
    assert rec["kernel_source_sha256"] == SHA
    assert rec["calibration"]["fetch_bytes_per_kib"] == pytest.approx(2048.0)
    assert rec["calibration"]["write_bytes_per_kib"] == pytest.approx(1024.0)
    bf16 = rec["legs"]["bf16"]
    assert bf16["dispatches"] == 3
    assert bf16["hbm_read_bytes_per_launch"] == pytest.approx(1100.0 * 2048.0)
    assert bf16["hbm_write_bytes_per_launch"] == pytest.approx(300.0 * 1024.0)
    assert bf16["hbm_bytes_per_launch"] == pytest.approx(1100.0 * 2048.0 + 300.0 * 1024.0)
    assert set(rec["legs"]) == {"bf16", "bf16_value_only", "fp32"}


def test_traffic_refuses_runs_of_different_sources(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(fetch, [(COPY, "FETCH_SIZE", 1.0), (BF16, "FETCH_SIZE", 1.0)])
    _write_counters(write, [(COPY, "WRITE_SIZE", 1.0), (BF16, "WRITE_SIZE", 1.0)])
    flog, wlog = tmp_path / "f.log", tmp_path / "w.log"
    flog.write_text(f"[bench] kernel source sha256 {SHA}\n")
    wlog.write_text(f"[bench] kernel source sha256 {'cd' * 32}\n")
    with pytest.raises(SystemExit):
        rs.main(["traffic", "--fetch", str(fetch), "--write", str(write), "--fetch-log",
                 str(flog), "--write-log", str(wlog), "--fetch-command", "cf",
                 "--write-command", "cw", "--copy-mib", "1", "--out", str(tmp_path / "t.json")])
