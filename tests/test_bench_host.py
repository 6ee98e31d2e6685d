"""Host-side arithmetic of bench.py (no GPU): the algorithmic flop count
F(p) against its term-by-term definition, the HBM and LDS rate fields of
the roofline object, the traffic summary's source-hash check, and the
refusal of more than one GPU."""

import json
import subprocess
import sys

import pytest

import bench


def test_flops_per_sample_terms():
    # F(p) = 2[2(p+1)^3 + 3(p+1)^2 + 4(p+1)] + 3[2p + 5p(p+1)/2 + 3(p+1)] + 50
    assert [bench.flops_per_sample(p) for p in (2, 3, 4)] == [320, 578, 959]
    # p = 3 term by term: contraction 2 x 192 FMA, basis 3 x 48, the rest 50
    assert bench.flops_per_sample(3) == 2 * 192 + 3 * 48 + 50


def test_rate_fields():
    h = bench.hbm_rate(1.2e8, 0.6)
    assert h["gb_per_s"] == pytest.approx(200.0)
    assert h["frac"] == pytest.approx(200.0 / 8000.0)
    assert bench.hbm_rate(None, 0.6) is None
    lds = bench.lds_rate(3, 1_000_000, 1.0)
    assert lds["bytes_per_sample"] == 4 * 64 + 32
    # bytes / (seconds x clock x compute units)
    assert lds["bytes_per_clk_per_cu"] == pytest.approx(288e6 / (1e-3 * 2.4e9 * 256))
    assert lds["frac"] == pytest.approx(lds["bytes_per_clk_per_cu"] / 128)


def test_traffic_needs_matching_sources(tmp_path, monkeypatch):
    rec = {"kernel_source_sha256": "0" * 64,
           "legs": {"bf16": {"hbm_bytes_per_launch": 1.0e8}}}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("bf16") is None
    rec["kernel_source_sha256"] = bench.kernel_source_hash()
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("bf16") == 1.0e8
    assert bench.measured_traffic("fp32") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=bench.ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
