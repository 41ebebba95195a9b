"""Host logic of bench.py (no GPU): counter CSV parsing and the copy
calibration, the traffic figures keyed by the kernel-source hash, the choice
of the dominant kernel class and the derived rates, and the one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY = "__amd_rocclr_copyBuffer"
KERN = "void lcc::k_bm_group<64, 512, 0, true>(lcc::AggArgs)"


def write_counter_csv(path, counter, rows):
    """A rocprofv3 counter-collection CSV with the columns the parser keys on."""
    cols = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": f"{value:.6f}"})


def test_counter_csv_groups_values_per_kernel(tmp_path):
    p = tmp_path / "fetch.csv"
    write_counter_csv(p, "FETCH_SIZE", [(COPY, 524288.0), (KERN, 10.0), (KERN, 30.0)])
    got = bench.read_counter_csv(str(p))
    assert got == {COPY: [524288.0], KERN: [10.0, 30.0]}


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path, capsys):
    # the 1 GiB copy reads as 524288 KiB of FETCH_SIZE (scale 2) and
    # 1048576 KiB of WRITE_SIZE (scale 1)
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counter_csv(f, "FETCH_SIZE", [(COPY, 524288.0), (KERN, 100.0), (KERN, 300.0)])
    write_counter_csv(w, "WRITE_SIZE", [(COPY, 1048576.0), (KERN, 8.0), (KERN, 8.0)])
    bench.pmc_summary(str(f), str(w))
    out = capsys.readouterr().out
    assert "scale 2.0000" in out and "scale 1.0000" in out
    row = next(line for line in out.splitlines() if "k_bm_group" in line)
    cells = [c.strip() for c in row.strip("|").split("|")]
    # mean 200 KiB fetched per dispatch, doubled; 8 KiB written
    assert cells[1] == "2"
    assert cells[2] == f"{200 * 1024 * 2:,}"
    assert cells[3] == f"{8 * 1024:,}"
    assert float(cells[4]) == pytest.approx((2 * 409600 + 2 * 8192) / 1e9, abs=1e-3)


def test_traffic_figures_follow_the_kernel_sources(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        entries = json.load(f)
    e = entries[-1]
    # figures taken on the sources of this hash are reported as they stand
    monkeypatch.setattr(bench, "kernel_source_sha1", lambda: e["source_sha1"])
    want = e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
    assert bench.measured_traffic(e["workload"], e["class"]) == want
    assert bench.measured_traffic(e["workload"], "no_such_class") is None
    # a change of the kernel sources makes the figures stale
    monkeypatch.setattr(bench, "kernel_source_sha1", lambda: "0" * 40)
    assert bench.measured_traffic(e["workload"], e["class"]) is None


def test_dominant_kernel_is_the_slowest_best_move_class():
    ks = {
        "bm_aggregate_g64_unit": {"ms": 100.0, "bytes": 8e11, "launches": 50},
        "bm_flat_seq_i32": {"ms": 120.0, "bytes": 6e11, "launches": 150},
        "cp_sort": {"ms": 500.0, "bytes": 1e12, "launches": 4},  # not a best-move class
        "bm_single_unit": {"ms": 20.0, "bytes": 1e11, "launches": 8},
    }
    r = bench.dominant_kernel(ks)
    assert r["kernel"] == "bm_flat_seq_i32"
    assert r["achieved"] == pytest.approx(6e11 / 0.120 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["avg_launch_ms"] == pytest.approx(0.8)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["traffic"] is None


def test_traffic_rate_uses_the_same_launch_time(monkeypatch):
    monkeypatch.setattr(bench, "copy_bandwidth_gbs", lambda dev: 5000.0)
    roof = {"achieved": 500.0, "traffic": 1.5e10, "avg_launch_ms": 2.5}
    out = bench.with_copy_peak(dict(roof), "cpu")
    assert out["frac_of_copy"] == pytest.approx(0.1)
    assert out["traffic_gbs"] == pytest.approx(1.5e10 / 2.5e-3 / 1e9)
    assert out["traffic_frac"] == pytest.approx(out["traffic_gbs"] / 8000.0)
    none = bench.with_copy_peak({"achieved": 500.0, "traffic": None, "avg_launch_ms": 2.5}, "cpu")
    assert "traffic_gbs" not in none


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
