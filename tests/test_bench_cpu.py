"""Host-side logic of the benchmark, on the CPU: the refusal of more than one GPU, and the
counter summaries built from rocprofv3 CSV traces (synthetic ones here, with known values) --
the calibration scales, the matrix-pipe occupancy and clock, the roofline block, and the
guard that drops a summary once the kernel's sources no longer match it."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _trace(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_scales_and_guard(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    gemm = "void hlb::crt_gemm_stream_kernel<hlb::CrtTile<4, 3, 2, 4> >(hlb::CrtGemmArgs)"
    copy = "__amd_rocclr_copyBuffer"
    # the 1 GiB calibration copy reads 512 MiB by the fetch counter and writes 1 GiB
    _trace(tmp_path / "f", [(copy, "FETCH_SIZE", 524288, 0, 1), (gemm, "FETCH_SIZE", 1000, 0, 1),
                            (gemm, "FETCH_SIZE", 3000, 0, 1), ("other", "FETCH_SIZE", 9e9, 0, 1)])
    _trace(tmp_path / "w", [(copy, "WRITE_SIZE", 1048576, 0, 1), (gemm, "WRITE_SIZE", 4000, 0, 1)])
    out = bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), 8192, 3, "crt_gemm")
    assert out["fetch_kib"] == 2000 and out["write_kib"] == 4000
    assert out["fetch_scale"] == 2.0 and out["write_scale"] == 1.0
    want = 2000 * 1024 * 2 + 4000 * 1024
    assert bench.measured_traffic("crt_gemm", 8192, 3) == want
    assert bench.measured_traffic("crt_gemm", 4096, 3) is None  # another workload
    rf = bench._roofline("crt_gemm", 10, 2.0, 5e12, 5, 8192, 3, 5000.0, "TOP/s", "int8 MAC x 2")
    # 2 launches per step: 2.5e12 ops per launch over 2 ms = 1250 TOP/s
    assert rf["achieved"] == pytest.approx(1250.0) and rf["frac"] == pytest.approx(0.25)
    assert rf["traffic"] == want and rf["traffic_gbs"] == pytest.approx(want / 2e-3 / 1e9)
    # a summary taken on other sources is not used
    path = bench.traffic_file("crt_gemm", 8192, 3)
    t = json.load(open(path))
    t["kernel_source_sha256"] = "0" * 64
    json.dump(t, open(path, "w"))
    assert bench.measured_traffic("crt_gemm", 8192, 3) is None
    assert bench._roofline("crt_gemm", 10, 2.0, 5e12, 5, 8192, 3, 5000.0, "TOP/s", "x")["traffic"] is None


def test_mfma_summary_occupancy_and_clock(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    gemm = "void hlb::gemm_i8_kernel<hlb::I8Tile<3, 7, 4, 2, 0>, false>(hlb::GemmArgs)"
    # two dispatches: 1000 cycles per XCD in 500 ns (2 GHz), half of the 1024 SIMDs' cycles busy
    rows = []
    for start in (0, 10_000):
        rows += [(gemm, "SQ_VALU_MFMA_BUSY_CYCLES", 1024 * 1000 * 0.5, start, start + 500),
                 (gemm, "GRBM_GUI_ACTIVE", 8 * 1000, start, start + 500),
                 (gemm, "SQ_BUSY_CYCLES", 123, start, start + 500)]
    _trace(tmp_path / "m", rows)
    out = bench.summarize_mfma(str(tmp_path / "m"), 8192, 3, "gemm_i8")
    assert out["dispatches"] == 2
    assert out["mfma_busy_frac"] == pytest.approx(0.5) and out["clock_ghz"] == pytest.approx(2.0)
    assert bench.measured_mfma("gemm_i8", 8192, 3) == {"busy_frac": pytest.approx(0.5),
                                                        "clock_ghz": pytest.approx(2.0)}
    assert bench.measured_mfma("gemm_i8", 16384, 2) is None
