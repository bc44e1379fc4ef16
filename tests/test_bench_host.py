"""Host-side checks of bench.py's output contract (no GPU)."""
import argparse
import os
import subprocess
import sys

import bench
from paper_1912_00539_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_measured_traffic_matches_the_current_kernel_sources():
    """The committed rocprofv3 traffic was taken on the kernels as they are now, so the bench line's
    roofline.traffic is reported (it becomes null once a measured kernel's source changes)."""
    h = bench.source_hash()
    for k in ("spmv", "spmv_resid", "factor_sweep_f32_async_fromA", "apply_bwd_last_f32_async", "stream_copy"):
        t = bench.load_traffic(k, h)
        assert t is not None and t > 0, k


def test_cpu_baseline_fields():
    c = W.case("quad32")
    r = bench.cpu_baseline(c, argparse.Namespace(apply_sweeps=3))
    assert r["kind"] == "oracle" and r["unit"] == "GB/s" and r["value"] > 0
    assert r["cores"] >= 1 and isinstance(r["sample"], str) and r["sample"]
    assert r["sequential"]["threads"] == 1 and r["sequential"]["ilu0_ms"] >= 0
