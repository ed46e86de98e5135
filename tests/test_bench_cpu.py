"""Host-side logic of bench.py (no GPU): the one-GPU guard, the lookup of
measured HBM traffic (valid only for the kernel source it was taken on) and
the per-class kernel table."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _write_profile(dirpath, entries):
    with open(os.path.join(dirpath, "x_traffic.md"), "w") as f:
        f.write("# traffic\n\n")
        for e in entries:
            f.write("traffic_json: " + json.dumps(e) + "\n")


def test_measured_traffic_only_for_the_current_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    src = bench.kernel_source_hash()
    good = {"kclass": "cgs_gram", "workload": "skyscraper3d", "kernel_source_sha256_16": src,
            "hbm_gb_per_launch": 1.4, "file": "x"}
    stale = dict(good, kernel_source_sha256_16="0" * 16, hbm_gb_per_launch=9.9)
    other = dict(good, kclass="spmm", hbm_gb_per_launch=1.2)
    _write_profile(tmp_path, [stale, other, good])
    assert bench.measured_traffic("cgs_gram", "skyscraper3d")["hbm_gb_per_launch"] == 1.4
    assert bench.measured_traffic("spmm", "skyscraper3d")["hbm_gb_per_launch"] == 1.2
    assert bench.measured_traffic("cgs_gram", "anisotropic3d") is None
    _write_profile(tmp_path, [stale])
    assert bench.measured_traffic("cgs_gram", "skyscraper3d") is None


def test_measured_traffic_per_row_order(tmp_path, monkeypatch):
    # lines without a row order are the domain order's; another row order
    # gets no traffic unless a line was measured with it
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    src = bench.kernel_source_hash()
    dom = {"kclass": "spmm", "workload": "randomblocks3d", "kernel_source_sha256_16": src,
           "hbm_gb_per_launch": 42.3, "file": "x"}
    _write_profile(tmp_path, [dom])
    assert bench.measured_traffic("spmm", "randomblocks3d")["hbm_gb_per_launch"] == 42.3
    assert bench.measured_traffic("spmm", "randomblocks3d", row_order="morton") is None
    _write_profile(tmp_path, [dom, dict(dom, row_order="morton", hbm_gb_per_launch=30.0)])
    assert bench.measured_traffic("spmm", "randomblocks3d", "fp64", "morton")["hbm_gb_per_launch"] == 30.0
    assert bench.measured_traffic("spmm", "randomblocks3d", "fp64", "domain")["hbm_gb_per_launch"] == 42.3


def test_kernel_source_hash_is_the_kernel_file():
    import hashlib
    path = os.path.join(ROOT, "paper_1804_10629_amd", "csrc", "ecg_kernels.hip")
    with open(path, "rb") as f:
        want = hashlib.sha256(f.read()).hexdigest()[:16]
    assert bench.kernel_source_hash() == want


def test_kernel_table_rates():
    stats = {"spmm": {"launches": 4, "ms": 1.0, "bytes": 4e9},
             "tsplit": {"launches": 0, "ms": 0.0, "bytes": 0.0}}
    t = bench.kernel_table(stats)
    assert set(t) == {"spmm"}
    assert abs(t["spmm"]["us_per_launch"] - 250.0) < 1e-9
    assert abs(t["spmm"]["gb_per_launch"] - 1.0) < 1e-9
    assert abs(t["spmm"]["gbs"] - 4000.0) < 1e-6
