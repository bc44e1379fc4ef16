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


def _stub_detail():
    """A result object shaped like the one bench.py builds on the GPU, with its long per-step arrays."""
    err = {"rel": 1.2345678901234567e-06, "max_block_rel": 5.678901234567891e-05}
    serve = {"solves_per_s": 2959.12, "elapsed_s": 0.676, "p50_ms": 2.57, "p99_ms": 8.88, "mean_ms": 3.08,
             "max_ms": 11.534, "converged": 2000, "max_rel_true_residual": 0.0008631065690128775, "mean_iters": 2.0,
             "solve_path_GBps": 4145.5, "ticks": 8000, "launches": 100000, "max_admitted": 200}
    steps = [{"step": t, "cfl": 10.0 * 1.5 ** t,
              "cold": {"ilu_residual": 0.01, "iters": 2, "converged": 1, "factor_ms": 0.3, "solve_ms": 0.5},
              "warm": {"ilu_residual": 0.001, "iters": 1, "converged": 1, "factor_ms": 0.3, "solve_ms": 0.5}}
             for t in range(12)]
    return {
        "metric": bench.METRIC, "value": 5589.1, "unit": "GB/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 4.306, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "tri2000: 2000x1000 quads split into 4000000 triangles, 15994000 4x4 blocks, CFL 100, "
                               "random permutation + RCM", "mode": "async", "build_sweeps": 1, "apply_sweeps": 3,
                   "fgmres_restart": 50, "rtol": 0.01, "factor_precision": "f32", "krylov_precision": "f64"},
        "roofline": {"bound": "hbm", "kernel": "spmv", "achieved": 5490.2, "peak": 8000.0, "unit": "GB/s",
                     "frac": 0.6863, "traffic": 2616000000, "launches": 60, "avg_launch_ms": 0.4342,
                     "algorithmic_bytes_per_launch": 2383208004},
        "frac_hbm_peak": 0.6986, "stream_copy_GBps": 5700.0, "frac_stream": 0.98, "factor_apply_GBps": 5600.0,
        "factor_sweeps_per_s": 1100.0, "solves_per_s": 232.2, "timing": "without per-launch profiling events",
        "fgmres_iters": [2] * 20, "ilu_residual": 0.004760681767857292, "converged": True,
        "max_rel_true_residual": 0.0007444273330686531,
        "kernels": {f"kernel_{q}": {"launches": 100, "ms": 1.0, "GBps": 5000.0} for q in range(40)},
        "compare": [{"mode": "sync", "fgmres_iters": [100] * 3}] * 2,
        "precision": {"f32_speedup_step": 1.6, "steps": {},
                      "f32_vs_f64": {k: {"sweeps1": {"X": err, "Dinv": err}, "sweeps2": {"X": err, "Dinv": err},
                                         "apply": err}
                                     for k in ("tri300_cfl100", "aniso1000_line", "aniso1000_rcm", "tri2000")}},
        "chunked": {"tri2000": {"chunk_over_async_step_time": 1.1}, "aniso1000_line": {"chunk_over_async_step_time": 0.9}},
        "configs": {"x": ["y" * 100] * 50},
        "orderings": {"x": ["y" * 100] * 50},
        "serving": {"saturation": {"batched_f32": serve, "one_at_a_time_f64": serve, "one_at_a_time_f32": serve},
                    "poisson": {"rate_per_s": 1096.0, "batched_f32": serve, "one_at_a_time_f64": serve},
                    "speedup_solves_per_s": 2.16,
                    "tight_tolerance": {"rtol": 1e-8, "requests": 400, "speedup_solves_per_s": 1.934,
                                        "batched_f32": dict(serve, max_iters=31),
                                        "one_at_a_time_f64": dict(serve, max_iters=30)}},
        "warm_start": {"totals": {"cold": {"iters": 24}, "warm": {"iters": 12}}, "steps": steps},
        "graphs": {k: {"n": 1024, "factor_sweeps": 3, "apply_sweeps": 3, "eager_us": 123.4, "graph_us": 56.7,
                       "speedup": 2.18, "replay_bits_equal": True} for k in ("quad32_f64", "tri300_f32")},
        "factor_convergence": {"summary": {k: {"D": 11085, "fixed_point_sweeps": 37,
                                               "f32_async_E_L": [0.03239, 0.001111, 4.155e-05, 1.88e-06, 7.728e-08],
                                               "f32_async_E_U": [0.08257, 0.002898, 0.000103, 3.774e-06, 1.348e-06]}
                                           for k in ("aniso1000_line", "tri2000")},
                               "runs": ["z" * 100] * 50},
        "cpu_baseline": {"value": 13.5, "unit": "GB/s", "cores": 16, "kind": "oracle", "cpu_model": "AMD EPYC 9575F",
                         "host_cpus": 256, "sample": "s" * 220, "seconds": 12.3,
                         "sequential": {"ilu0_ms": 615.0, "exact_substitution_ms": 80.0, "threads": 1, "what": "w" * 200},
                         "oracle_check": {"what": "w" * 80, "f64_bitwise_equal": True,
                                          "f64": {"X": err, "Dinv": err}, "f32": {"X": err, "Dinv": err}}},
        "source_hash": "0123456789abcdef",
    }


def test_headline_line_is_compact_and_parseable(tmp_path, capsys):
    """The last stdout line (the one the driver parses) stays well under its 8,000-character tail and
    carries the headline; the full object goes to the detail file."""
    import json
    out = _stub_detail()
    path = str(tmp_path / "detail.json")
    bench.emit(out, path)
    lines = capsys.readouterr().out.strip().splitlines()
    last = lines[-1]
    assert len(last) < 3900, len(last)   # a margin below 4 KB for longer figures of a real run
    h = json.loads(last)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "serving", "value_covers",
              "frac_stream", "factor_apply_GBps", "precision"):
        assert k in h, k
    assert h["config"]["workload"].startswith("tri2000")
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in h["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in h["cpu_baseline"], k
    assert h["serving"]["saturation"]["batched_f32"]["p99_ms"] == 8.88
    assert h["serving"]["tight"]["rtol"] == 1e-8 and h["serving"]["tight"]["speedup"] == 1.934
    assert h["precision"]["f32_vs_f64"]["tri2000"]["z"][1] > 0
    assert json.load(open(path)) == out
