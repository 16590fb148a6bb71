"""bench.py on the host: the single-GPU guard and the committed HBM counter
records (each is reported only while it matches the kernel sources it was
taken on)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("path,sources,workload", [
    (bench.TRAFFIC_FILE, ("gemm.hip", "common.h"), "dense-65536x65536-k50-hals-f32"),
    (bench.TRAFFIC_FILE_CSR, bench.SPARSE_SOURCES, "csr-1048576x1048576-d1e-4-k50-abpp-f32"),
    (bench.TRAFFIC_FILE_FP8, bench.LOWP_SOURCES, "dense-131072x65536-k100-hals-fp8"),
    (bench.TRAFFIC_FILE_BF16, bench.LOWP_SOURCES, "dense-131072x65536-k100-hals-bf16"),
])
def test_traffic_records_match_the_current_kernels(path, sources, workload):
    with open(path) as f:
        rec = json.load(f)
    assert rec["kernel_source_hash"] == bench.kernel_source_hash(sources)
    t = bench.load_traffic(bench.kernel_source_hash(sources), path, workload)
    assert t is not None and t["hbm_bytes_per_launch"] > 0
    # a record taken on other sources is not reported
    assert bench.load_traffic("0" * 16, path, workload) is None
