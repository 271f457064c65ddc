"""Host logic of bench.py (no GPU): the one-GPU guard, the traffic summary built from rocprofv3 counter CSVs (each
counter scaled by its reading for a copy of known size), the rule that traffic is null once the kernel sources
differ from those the counters were taken with, and the kernel-stats table."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KEY = "k_digest<2, 1, 2, 0, false, 1>"


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for disp, name, value in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_scales_by_the_copy(tmp_path):
    gib_kib = float(1 << 20)
    copy = "__amd_rocclr_copyBuffer(char const*, char*)"
    kern = "void uqc::" + KEY + "(uqc::TaskDev const*, long long const*, int, long long, long long)"
    # the copy moves 1 GiB each way; its FETCH_SIZE reads half of that (scale 2), WRITE_SIZE all of it (scale 1)
    _counter_csv(tmp_path / "cf.csv", "FETCH_SIZE", [(1, copy, gib_kib / 2)])
    _counter_csv(tmp_path / "cw.csv", "WRITE_SIZE", [(1, copy, gib_kib)])
    # two launches of the class kernel, counters split over two rows each (summed per dispatch)
    _counter_csv(tmp_path / "kf.csv", "FETCH_SIZE", [(7, kern, 100.0), (7, kern, 50.0), (9, kern, 150.0)])
    _counter_csv(tmp_path / "kw.csv", "WRITE_SIZE", [(7, kern, 30.0), (9, kern, 10.0)])
    out = tmp_path / "traffic.json"
    doc = bench.summarize_pmc(str(tmp_path / "kf.csv"), str(tmp_path / "kw.csv"), str(tmp_path / "cf.csv"),
                              str(tmp_path / "cw.csv"), str(out), "cmd")
    assert doc["copy_kernel"] == "__amd_rocclr_copyBuffer"
    assert doc["fetch_scale"] == pytest.approx(2.0) and doc["write_scale"] == pytest.approx(1.0)
    k = doc["kernels"][KEY]
    assert k["launches"] == 2
    assert k["fetch_bytes_per_launch"] == pytest.approx(150.0 * 2.0 * 1024)
    assert k["write_bytes_per_launch"] == pytest.approx(20.0 * 1.0 * 1024)
    assert json.load(open(out))["kernel_sources_sha256"] == bench.kernel_sources_sha256()


def test_traffic_is_null_when_the_kernel_sources_differ(tmp_path, monkeypatch):
    doc = {"kernel_sources_sha256": bench.kernel_sources_sha256(),
           "kernels": {KEY: {"fetch_bytes_per_launch": 3.0, "write_bytes_per_launch": 4.0, "launches": 1},
                       "k_digest_team<2, 2, 2, 2, false, 1>": {"fetch_bytes_per_launch": 5.0,
                                                               "write_bytes_per_launch": 6.0, "launches": 1}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.traffic_for(KEY) == 7.0
    # a team class is looked up under its team kernel's name
    assert bench.traffic_for(bench.dom_kernel_key(2222)) == 11.0
    assert bench.traffic_for(bench.dom_kernel_key(1111)) is None
    doc["kernel_sources_sha256"] = "0" * 64
    p.write_text(json.dumps(doc))
    assert bench.traffic_for(KEY) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.traffic_for(KEY) is None


def test_kernel_source_hash_covers_the_kernels_and_not_host_files():
    csrc = os.path.join(ROOT, "paper_1303_4916_amd", "csrc")
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(csrc, f)), f
    assert "uqc_api.cpp" not in bench.KERNEL_SOURCES and "uqc_serve.cpp" not in bench.KERNEL_SOURCES
    assert len(bench.kernel_sources_sha256()) == 64


def test_kernel_stats_table(tmp_path):
    p = tmp_path / "stats.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "void uqc::k_zero(double*, unsigned long)", "Calls": 4, "AverageNs": 1000,
                    "TotalDurationNs": 4000, "Percentage": 0.1})
        w.writerow({"Name": "void uqc::" + KEY + "(uqc::TaskDev const*)", "Calls": 2, "AverageNs": 8.5e6,
                    "TotalDurationNs": 1.7e7, "Percentage": 99.9})
    out = tmp_path / "stats.md"
    bench.summarize_stats(str(p), str(out), "rocprofv3 ... -- python3 bench.py", "title")
    lines = out.read_text().splitlines()
    rows = [ln for ln in lines if ln.startswith("| k_")]
    assert rows[0] == "| %s | 2 | 8.500 | 17.00 | 99.9 |" % KEY
    assert rows[1] == "| k_zero | 4 | 0.001 | 0.00 | 0.1 |"
    assert "rocprofv3 ... -- python3 bench.py" in lines
