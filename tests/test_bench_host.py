"""Host logic of bench.py (CPU only): the one-GPU refusal, the hash-guarded
traffic figure and the rocprofv3 summarisers, on small hand-made CSV files
whose expected figures are computed by hand here."""
import csv
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_figure_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {64: str(f), 32: str(tmp_path / "none.txt")})
    assert bench.read_traffic() is None                      # absent
    f.write_text(f"# comment: 1\nkernel_source_sha256_16: {bench.kernel_sha()}\n"
                 "hbm_bytes_per_launch: 1234.0\n")
    assert bench.read_traffic() == 1234.0
    f.write_text("kernel_source_sha256_16: 0000000000000000\nhbm_bytes_per_launch: 1234.0\n")
    assert bench.read_traffic() is None                      # taken on another source
    f.write_text(f"kernel_source_sha256_16: {bench.kernel_sha()}\nhbm_bytes_per_launch: n/a\n")
    assert bench.read_traffic() is None                      # unreadable figure


def test_summarize_traffic_scales_by_the_copy_calibration(tmp_path):
    n_u = 1000                      # the calibration copy moves 4 n_u = 4000 bytes each way
    roof = f"void stk::{bench.ROOF_KERNEL}(stk::LevelDev, ...)"
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    dF, dW = tmp_path / "F", tmp_path / "W"
    dF.mkdir()
    dW.mkdir()
    # FETCH_SIZE reads 2x the known bytes on the copy (scale 0.5); the roofline
    # kernel's largest grid reads 10 and 14 KiB on two launches (average 12)
    _write_csv(dF / "run_counter_collection.csv", hdr, [
        ["__amd_rocclr_copyBuffer", 4096, "FETCH_SIZE", 8000 / 1024],
        [roof, 6144, "FETCH_SIZE", 10.0],
        [roof, 6144, "FETCH_SIZE", 14.0],
        [roof, 1536, "FETCH_SIZE", 99.0],
    ])
    # WRITE_SIZE reads exactly the known bytes (scale 1); the kernel writes 3 KiB
    _write_csv(dW / "run_counter_collection.csv", hdr, [
        ["__amd_rocclr_copyBuffer", 4096, "WRITE_SIZE", 4000 / 1024],
        [roof, 6144, "WRITE_SIZE", 3.0],
    ])
    out = tmp_path / "traffic.txt"
    bench.summarize_traffic(str(dF), str(dW), n_u, str(out), ("cmdF", "cmdW"))
    kv = dict(line.split(": ", 1) for line in out.read_text().splitlines() if not line.startswith("#"))
    assert float(kv["fetch_scale"]) == pytest.approx(0.5)
    assert float(kv["write_scale"]) == pytest.approx(1.0)
    assert float(kv["fetch_bytes_per_launch"]) == pytest.approx(12 * 1024 * 0.5, abs=1)
    assert float(kv["write_bytes_per_launch"]) == pytest.approx(3 * 1024, abs=1)
    assert float(kv["hbm_bytes_per_launch"]) == pytest.approx(12 * 512 + 3 * 1024, abs=1)
    assert kv["kernel_source_sha256_16"] == bench.kernel_sha()


def test_summarize_counters_averages_per_kernel_and_grid(tmp_path):
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    _write_csv(tmp_path / "run_counter_collection.csv", hdr, [
        ["void stk::k_transfer<float, 1>(x)", 1000, "LdsUtil", 30.0],
        ["void stk::k_transfer<float, 1>(x)", 1000, "LdsUtil", 40.0],
        ["void stk::k_transfer<float, 1>(x)", 10, "LdsUtil", 5.0],
        ["void stk::k_other(x)", 1000, "LdsUtil", 99.0],
    ])
    out = tmp_path / "c.txt"
    bench.summarize_counters(str(tmp_path), str(out), "the command", "k_transfer")
    lines = out.read_text().splitlines()
    assert lines[1] == "# command: the command"
    body = [l for l in lines if "k_transfer" in l]
    assert len(body) == 2 and not any("k_other" in l for l in lines)
    big = [l for l in body if "grid       1000" in l][0]
    assert float(big.split()[-3]) == pytest.approx(35.0) and "(2 dispatches)" in big


def test_summarize_profile_groups_the_roofline_kernel_by_grid(tmp_path):
    roof = f"void stk::{bench.ROOF_KERNEL}(stk::LevelDev, ...)"
    _write_csv(tmp_path / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"], [
        [roof, 3, 9000, 3000, 75.0],
        ["void stk::k_other(x)", 1, 3000, 3000, 25.0],
    ])
    _write_csv(tmp_path / "run_kernel_trace.csv", ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"], [
        [roof, 6144, 0, 4000],
        [roof, 6144, 10000, 12000],
        [roof, 1536, 20000, 23000],
        ["void stk::k_other(x)", 6144, 0, 3000],
    ])
    out = tmp_path / "p.txt"
    bench.summarize_profile(str(tmp_path), str(out), "cmd")
    text = out.read_text()
    assert "total kernel time 0.000 s over 2 kernels" in text
    assert "grid       6144:      2 launches, average        3.0 us" in text
    assert "grid       1536:      1 launches, average        3.0 us" in text


def test_roofline_fields():
    """The roofline object: algorithmic flops of the launch over its time
    against the FP64 (or FP32) peak, algorithmic bytes over HBM."""
    r = bench._roofline(64, 1000, 300, 20, 2.0, None)
    flops = bench.A_FLOPS_PER_TET * 1000
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_FP64_TFLOPS
    assert r["achieved"] == pytest.approx(flops / 2e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert r["hbm_gbs_algorithmic"] == pytest.approx((2 * 300 + 20) * 8 / 2e-3 / 1e9)
    r32 = bench._roofline(32, 1000, 300, 20, 2.0, 4960.0)
    assert r32["peak"] == bench.PEAK_FP32_TFLOPS and r32["traffic_over_algorithmic"] == pytest.approx(2.0)


def test_flop_figure_is_checked_against_the_sweep_source(tmp_path, monkeypatch):
    """The flop count per micro-tet is reported as checked only when the
    counter summary was taken on the current sweep source; the summariser
    divides the executed-flop counters of the largest grid by the micro-tets."""
    f = tmp_path / "flops.txt"
    monkeypatch.setattr(bench, "FLOPS_FILE", str(f))
    assert bench.read_flops() == (bench.A_FLOPS_PER_TET, False)
    d = tmp_path / "pmc"
    d.mkdir()
    k64 = f"void stk::{bench.ROOF_KERNELS[64]}(stk::LevelDev, ...)"
    k32 = f"void stk::{bench.ROOF_KERNELS[32]}(stk::LevelDev, ...)"
    _write_csv(d / "run_counter_collection.csv", ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], [
        [k64, 6144, "SQ_INSTS_VALU_FLOPS_FP64", 130000.0],
        [k64, 6144, "SQ_INSTS_VALU_FLOPS_FP64", 132000.0],
        [k64, 1536, "SQ_INSTS_VALU_FLOPS_FP64", 99.0],
        [k32, 6144, "SQ_INSTS_VALU_FLOPS_FP32", 120000.0],
    ])
    bench.summarize_flops(str(d), 100, str(f), "cmd")
    kv = bench._kv(str(f))
    assert kv["executed_flops_per_micro_tet_fp64"].startswith("1310.0")
    assert kv["executed_flops_per_micro_tet_fp32"].startswith("1200.0")
    assert bench.read_flops() == (bench.A_FLOPS_PER_TET, True)
    f.write_text("kernel_source_sha256_16: 0000000000000000\n")
    assert bench.read_flops() == (bench.A_FLOPS_PER_TET, False)


def test_sweep_hash_ignores_kernels_outside_the_sweep(tmp_path, monkeypatch):
    """A change after the sweep (another kernel) keeps the hash; a change in
    the sweep's source changes it."""
    src = open(bench.KERNEL_SRC).read()
    base = bench.kernel_sha()
    k = tmp_path / "k.hip"
    monkeypatch.setattr(bench, "KERNEL_SRC", str(k))
    k.write_text(src + "\n// another kernel\n")
    assert bench.kernel_sha() == base
    i = src.index("k_sweep(")
    k.write_text(src[:i] + " " + src[i:])
    assert bench.kernel_sha() != base
