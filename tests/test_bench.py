"""Host-side logic of bench.py (no GPU): the one-GPU contract, the
copy-calibrated HBM traffic summary of rocprofv3 counter runs, and the guard
that reports no traffic for a kernel source other than the profiled one."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KERNEL = "void gcp::k_gemm16<5>(gcp::GemmArgs)"
COPY = "__amd_rocclr_copyBuffer"
STREAM = "gcp::k_stream_lds(unsigned short const*)"


def _write_counters(d, counter, rows):
    """One rocprofv3 counter_collection.csv with (kernel name, KiB) rows."""
    os.makedirs(os.path.join(d, "node"), exist_ok=True)
    with open(os.path.join(d, "node", "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.fixture
def sandbox(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "product_kernel_hash", lambda: "source-a")
    return tmp_path


def test_pmc_summary_scales_each_counter_by_its_yardstick(sandbox):
    copy_kib = bench.COPY_BYTES / 1024
    # FETCH_SIZE is scaled by the global-to-LDS stream of known size (here it
    # reads half of its true bytes), WRITE_SIZE by the copy (all of them);
    # launches that did no work (past a solve's stop) are left out
    _write_counters(sandbox / "fetch", "FETCH_SIZE",
                    [(KERNEL, 3.0e6), (KERNEL, 3.2e6), (KERNEL, 0.0), (STREAM, 0.5 * copy_kib),
                     (COPY, 0.7 * copy_kib), ("other", 9e9)])
    _write_counters(sandbox / "write", "WRITE_SIZE",
                    [(KERNEL, 4.0e5), (KERNEL, 6.0e5), (COPY, copy_kib)])
    assert bench.summarize_pmc("fp16x3", 1, str(sandbox / "fetch"), str(sandbox / "write")) == 0
    d = json.load(open(sandbox / "profiles" / "gemm_fp16x3_M8192_pmc.json"))
    assert d["kernel"] == "k_gemm16<5>" and d["kernel_source_sha256"] == "source-a"
    assert d["FETCH_SIZE"]["launches"] == 2
    assert d["FETCH_SIZE"]["factor"] == pytest.approx(0.5)
    assert d["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(3.1e6 * 1024 / 0.5)
    assert d["WRITE_SIZE"]["factor"] == pytest.approx(1.0)
    assert d["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(5.0e5 * 1024)
    assert d["hbm_bytes_per_launch"] == pytest.approx(3.1e6 * 1024 / 0.5 + 5.0e5 * 1024)
    # the summary is used while the kernel source is the profiled one, and only then
    assert bench.pmc_traffic("gemm_fp16x3_M8192") == pytest.approx(d["hbm_bytes_per_launch"])
    bench.product_kernel_hash = lambda: "source-b"
    assert bench.pmc_traffic("gemm_fp16x3_M8192") is None
    assert bench.pmc_traffic("gemm_bf16x6_M8192") is None


def test_pmc_summary_needs_the_yardsticks(sandbox):
    # without the calibration kernels no scale factor exists: the summary
    # fails instead of guessing
    _write_counters(sandbox / "fetch", "FETCH_SIZE", [(KERNEL, 3.0e6), (COPY, 10.0)])
    _write_counters(sandbox / "write", "WRITE_SIZE", [(KERNEL, 4.0e5)])
    assert bench.summarize_pmc("fp16x3", 1, str(sandbox / "fetch"), str(sandbox / "write")) == 1
    assert not (sandbox / "profiles" / "gemm_fp16x3_M8192_pmc.json").exists()


def test_product_kernel_hash_covers_the_kernel_source():
    h = bench.product_kernel_hash()
    assert len(h) == 64 and h == bench.product_kernel_hash()
