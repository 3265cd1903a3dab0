"""Host-side pieces of bench.py (no GPU): the SpMM kernel names it matches
against rocprofv3 traces, the committed HBM-traffic record it reports, and
the one-GPU refusal."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("args,name", [
    (("double", 1, 4, 0), "k_filter_spmm<double, 1, 4, false, false, false>"),
    (("double", 1, 4, 2 | 4), "k_filter_spmm<double, 1, 4, true, false, true>"),
    (("float", 4, 4, 1), "k_filter_spmm<float, 4, 1, false, true, false>"),
    (("double", 2, 4, 8), "k_filter_spmm_paired<double, 2, 2, 3, false, false>"),
    (("double", 1, 2, 8 | 16 | 4), "k_filter_spmm_paired<double, 1, 2, 1, false, true>"),
    (("float", 4, 8, 8 | 1), "k_filter_spmm_paired<float, 4, 2, 3, true, false>"),
    (("double", 1, 1, 32), "k_filter_spmm_grid<double, 1, 8, 8, false, false>"),
    (("float", 1, 2, 32 | 64 | 4), "k_filter_spmm_grid<float, 2, 64, 1, false, true>"),
])
def test_spmm_kernel_names(args, name):
    assert bench.spmm_kernel_name(*args) == name


def test_traffic_record_matches_source_and_kernels():
    lines = open(bench.TRAFFIC_FILE).read().splitlines()
    rec = json.loads(next(l.split(":", 1)[1] for l in lines if l.startswith("traffic-json:")))
    sha = bench.spmm_source_sha256()
    for kern, k in rec["kernels"].items():
        t = bench.measured_traffic(kern)
        if rec["spmm_source_sha256"] == sha:
            assert t == pytest.approx(1024.0 * (k["fetch_kib"] * rec["copy_fetch_factor"] +
                                                k["write_kib"] * rec["copy_write_factor"]))
        else:  # counters taken on another version of the kernel: not reported
            assert t is None
    assert bench.measured_traffic("k_filter_spmm<double, 1, 1, false, false, false>") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
