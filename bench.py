#!/usr/bin/env python
"""Benchmark of the asynchronous block-ILU(0) hot path on one MI355X.

One step = factorisation (init + build sweeps) + a restarted FGMRES solve to rtol from x0 = 0,
right-preconditioned by the sweep apply (apply sweeps forward + backward per iteration), on the
4,000,000-cell split-quad triangle mesh (2000 x 1000 quads, 15,994,000 4x4 blocks, CFL 100,
random permutation + reverse Cuthill-McKee). Factor and sweeps in FP32, Krylov in FP64.

value = algorithmic bytes of every kernel of the step / wall time of the step (GB/s); the byte
counts come from the library (one figure per launch, every array element counted once), in a
profiled run; the wall time is that of the same steps run again without the per-launch events
(the same work: identical iteration counts, else the profiled time is used).

The "serving" object measures the continuous-batching server on a stream of independent solves
(FP32 preconditioner, batched launches) against one-solve-at-a-time FP64 on the same stream:
solves/s at saturation and p50/p99 latency under Poisson arrivals. The "precision" object runs the
same step with the preconditioner in FP64, and gives the distance between the FP32 and FP64 factors.
The "chunked" object compares the chunked (Gauss-Seidel within chunks) sweeps with the unchunked
asynchronous ones on the same step, and on the line-ordered anisotropic mesh.
The "orderings" object measures the step under the orderings of Section 5 (RCM, one-way
dissection, lines of anisotropic cells, line and hybrid line-X orderings).
The "configs" object gives factor and apply bandwidth on the 180,000-triangle and the
500,000-cell anisotropic workloads (line and RCM order), SYNC/ASYNC, FP32/FP64.
The full result object goes to a detail file (--detail) and to stderr; the last line of stdout is a
compact headline of a few KB (the figures above and a summary of each sub-benchmark).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "ABILU factor+apply GB/s (% HBM peak); batched FGMRES solves/s + p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources of the single-system kernels the measured traffic belongs to (the serving, setup and
# generator sources do not enter them).
KERNEL_SOURCES = ("abilu_internal.h", "kernels.h", "apply.hip", "factor.hip", "krylov.hip", "api.hip")


def source_hash():
    """Hash of the measured kernels' sources with comments and blank lines removed."""
    import re
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1912_00539_amd", "csrc")
    for f in KERNEL_SOURCES:
        text = open(os.path.join(d, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(f.encode() + b"\0" + text.encode())
    return h.hexdigest()[:16]


def run_steps(sysm, args, mode, steps, profile, build_sweeps=None, maxit=None):
    import torch
    from paper_1912_00539_amd import abilu as L
    results = []
    nb = args.build_sweeps if build_sweeps is None else build_sweeps
    if profile:
        L.abilu_profile_enable(True, 200000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sysm.factor(nb, mode)
        st, res = sysm.solve(apply_sweeps=args.apply_sweeps, mode=mode, rtol=args.rtol,
                             maxit=args.maxit if maxit is None else maxit, restart=args.restart)
        results.append((st, res))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = None
    if profile:
        rep = L.abilu_profile_report()
        L.abilu_profile_enable(False)
    return t1 - t0, results, rep


def stream_reference(nbytes=2 << 30, reps=5):
    """Achievable HBM copy bandwidth with the library's STREAM copy kernel (read + write)."""
    import torch
    from paper_1912_00539_amd import abilu as L
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    L.abilu_stream_copy(b, a, nbytes)
    torch.cuda.synchronize()
    L.abilu_profile_enable(True, 64)
    for _ in range(reps):
        L.abilu_stream_copy(b, a, nbytes)
    rep = L.abilu_profile_report()
    L.abilu_profile_enable(False)
    cnt, ms, by = rep["stream_copy"]
    del a, b
    torch.cuda.empty_cache()
    return by / (ms / 1e3) / 1e9


def oracle_bytes_f64(N, Z, ZL, ZU, P, apply_sweeps):
    """Algorithmic bytes of the oracle sample (FP64 everywhere): one sweep, apply, SpMV."""
    sF = 8.0
    sweep = 4 * (N + 1) + 4 * N + 4 * ZL + 4 * (Z + 1) + 8 * P + 128 * Z + 16 * sF * min(2 * P, Z) + 32 * sF * N + 16 * sF * Z
    fwd = 8 * N + 4 * ZL + 16 * sF * ZL + 32 * N + 4 * N * sF + 4 * N * sF
    bwd = 8 * N + 4 * ZU + 16 * sF * ZU + 4 * N * sF * 3 + 16 * sF * N
    spmv = 4 * (N + 1) + 4 * Z + 128 * Z + 64 * N
    return sweep + apply_sweeps * (fwd + bwd) + spmv


def gpu_sync_factors(case):
    """One synchronous factor sweep from A on the GPU in FP64 and FP32, as (X in CSR block order,
    Dinv) float64 host arrays, for the check against the oracle in cpu_baseline."""
    import torch
    from paper_1912_00539_amd.runtime import DeviceSystem
    out = {}
    for prec in ("f64", "f32"):
        s = DeviceSystem(case, prec=prec, restart=1)
        s.factor(1, "sync")
        out[prec] = s.factor_host()
        del s
        torch.cuda.empty_cache()
    return out


def cpu_baseline(case, args, gpu=None):
    """The oracle as it stands, on the host cores, on a bounded sample of the same workload. With
    `gpu` (gpu_sync_factors), the oracle's one-sweep factor of the first sample is also compared
    with the GPU's: FP64 bit for bit, FP32 as relative errors."""
    import numpy as np
    import oracle
    n, rp, ci, A = case.n, case.rowptr, case.colidx, case.vals
    ptr, pik, pkj = oracle.pairs(n, rp, ci)
    P = int(ptr[-1])
    Z = case.nnzb
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    ZL = int(np.count_nonzero(ci < rows))
    ZU = Z - n - ZL
    reps = 0
    check = None
    t0 = time.perf_counter()
    while reps < 50 and (reps == 0 or time.perf_counter() - t0 < 10.0):
        X, D, _ = oracle.factor_sync(n, rp, ci, A, 1)
        if reps == 0 and gpu:
            tc = time.perf_counter()
            check = oracle_check(X, D, gpu)
            t0 += time.perf_counter() - tc   # the comparison is not oracle work
        z = oracle.apply_sync(n, rp, ci, X, D, case.b, args.apply_sweeps)
        oracle.spmv(n, rp, ci, A, z)
        reps += 1
    t1 = time.perf_counter()
    by = reps * oracle_bytes_f64(n, Z, ZL, ZU, P, args.apply_sweeps)
    # the sequential reference: traditional block ILU(0) and exact block substitutions, one thread
    s0 = time.perf_counter()
    Xs, Ds, _ = oracle.ilu0_seq(n, rp, ci, A)
    s1 = time.perf_counter()
    oracle.trisolve_exact(n, rp, ci, Xs, Ds, case.b)
    s2 = time.perf_counter()
    del Xs, Ds
    cpu_model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(by / (t1 - t0) / 1e9, 3), "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model, "host_cpus": os.cpu_count(),
            "sample": f"{reps} x (1 SYNC FP64 factor sweep + {args.apply_sweeps} apply sweep pairs + 1 SpMV) on the "
                      f"full {n}-cell matrix ({t1 - t0:.1f} s); bytes by the GPU kernels' model, in FP64",
            "seconds": round(t1 - t0, 2), "oracle_check": check,
            "sequential": {"ilu0_ms": round((s1 - s0) * 1e3, 1), "exact_substitution_ms": round((s2 - s1) * 1e3, 1),
                           "threads": 1, "what": "traditional block ILU(0) (row by row) and the exact forward and "
                                                 "backward block substitutions, once each, on the full matrix"}}


def oracle_check(X, D, gpu):
    """GPU one-sweep synchronous factors against the oracle's (X, D): FP64 bitwise equality and the
    largest relative difference; FP32 relative Frobenius and largest per-block relative errors."""
    import numpy as np

    def errs(a, ref):
        d = (a - ref).reshape(len(ref), -1)
        rn = np.linalg.norm(ref.reshape(len(ref), -1), axis=1)
        dn = np.linalg.norm(d, axis=1)
        nz = rn > 0
        return {"rel": float(f"{np.linalg.norm(d) / np.linalg.norm(ref):.3e}"),
                "max_block_rel": float(f"{(dn[nz] / rn[nz]).max() if nz.any() else 0.0:.3e}")}
    out = {"what": "one synchronous factor sweep from A on the full matrix, GPU against the oracle"}
    if "f64" in gpu:
        Xg, Dg = gpu["f64"]
        out["f64_bitwise_equal"] = bool(np.array_equal(Xg, X) and np.array_equal(Dg, D))
        out["f64"] = {"X": errs(Xg, X), "Dinv": errs(Dg, D)}
    if "f32" in gpu:
        Xg, Dg = gpu["f32"]
        out["f32"] = {"X": errs(Xg, X), "Dinv": errs(Dg, D)}
    return out


def load_traffic(kernel, shash):
    """Measured bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated) recorded under
    profiles/ for this kernel, or None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_tri2000_async_f32.txt")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    e = t.get(kernel)
    if not e or e.get("source_hash") != shash:
        return None
    return e.get("bytes_per_launch")


def percentiles(lat):
    import numpy as np
    a = np.asarray(lat, dtype=np.float64)
    return {"p50_ms": round(float(np.percentile(a, 50)) * 1e3, 3), "p99_ms": round(float(np.percentile(a, 99)) * 1e3, 3),
            "mean_ms": round(float(a.mean()) * 1e3, 3), "max_ms": round(float(a.max()) * 1e3, 3)}


def serving_bench(args):
    """Continuous batching (FP32 preconditioner, FP64 Krylov, batched launches) against the plain
    one-solve-at-a-time FP64 form, on the same request stream: saturation (all released at t = 0)
    and Poisson arrivals at 0.8 x the one-at-a-time throughput."""
    import numpy as np
    import torch
    from paper_1912_00539_amd import abilu as L
    from paper_1912_00539_amd import workloads as W
    reqs = W.serving_requests(args.serve_requests, seed=args.serve_seed)
    common = dict(mode="async", factor_sweeps=args.build_sweeps, apply_sweeps=args.apply_sweeps, restart=30,
                  maxit=300, rtol=args.rtol)
    forms = {"batched_f32": L.serve_config(prec="f32", max_active=args.serve_slots, **common),
             "one_at_a_time_f64": L.serve_config(prec="f64", max_active=1, **common),
             "one_at_a_time_f32": L.serve_config(prec="f32", max_active=1, **common)}
    forms = {k: v for k, v in forms.items() if k in args.serve_forms.split(",")}
    pool = torch.empty(int(args.serve_pool_gib * 2**30) // 256 * 256, dtype=torch.uint8, device="cuda")
    warm = W.serving_requests(8, seed=args.serve_seed + 1)
    for cfg in forms.values():
        srv = L.Server(cfg, pool)
        srv.run(warm)
        srv.destroy()

    def run(name, arrivals):
        srv = L.Server(forms[name], pool)
        res, el = srv.run(reqs, arrivals=arrivals)
        stats = srv.stats()
        srv.destroy()
        lat = [r["t_done"] - r["t_arrival"] for r in res]
        ok = sum(1 for r in res if r["converged"] and r["rel_true_residual"] <= args.rtol)
        out = {"solves_per_s": round(len(reqs) / el, 2), "elapsed_s": round(el, 3), **percentiles(lat),
               "converged": ok, "max_rel_true_residual": max(r["rel_true_residual"] for r in res),
               "mean_iters": round(float(np.mean([r["iters"] for r in res])), 2),
               "solve_path_GBps": round(stats["bytes"] / el / 1e9, 1), "ticks": stats["ticks"],
               "launches": stats["launches"], "max_admitted": None}
        ev = sorted([(r["t_admit"], 1) for r in res] + [(r["t_done"], -1) for r in res], key=lambda e: (e[0], e[1]))
        cur = peak = 0
        for _, d in ev:
            cur += d
            peak = max(peak, cur)
        out["max_admitted"] = peak
        log(f"serving {name}: {out}")
        return out

    sat = {name: run(name, None) for name in forms}
    kernel_profile = None
    if "batched_f32" in forms and args.serve_profile:
        # the same saturation run again with a HIP event pair around every batched launch: each
        # kernel's bandwidth against the sum of its members' algorithmic bytes
        srv = L.Server(forms["batched_f32"], pool)
        L.abilu_profile_enable(True, 400000)
        srv.run(reqs)
        rep = L.abilu_profile_report()
        L.abilu_profile_enable(False)
        srv.destroy()
        kernel_profile = {k: {"launches": v[0], "ms": round(v[1], 3), "GB": round(v[2] / 1e9, 2),
                              "GBps": round(v[2] / (v[1] / 1e3) / 1e9, 1) if v[1] > 0 else None}
                          for k, v in sorted(rep.items(), key=lambda kv: -kv[1][1]) if not k.startswith("_")}
        log(f"serving kernel profile (batched_f32): {kernel_profile}")
    poisson, lam = {}, None
    if "one_at_a_time_f64" in sat and not args.serve_saturation_only:
        lam = 0.8 * sat["one_at_a_time_f64"]["solves_per_s"]
        u = W.uniform01(args.serve_seed, 14, np.arange(len(reqs), dtype=np.int64))
        arrivals = np.cumsum(-np.log1p(-u) / lam)
        poisson = {name: run(name, arrivals) for name in forms if name != "one_at_a_time_f32"}
    poisson_high = None
    if "batched_f32" in sat and not args.serve_saturation_only:
        # the batched server at 0.8 x its own saturation rate (a load the one-at-a-time forms cannot carry)
        lam_hi = 0.8 * sat["batched_f32"]["solves_per_s"]
        u = W.uniform01(args.serve_seed, 15, np.arange(len(reqs), dtype=np.int64))
        poisson_high = {"rate_per_s": round(lam_hi, 2), "batched_f32": run("batched_f32", np.cumsum(-np.log1p(-u) / lam_hi))}
    tight = None
    if args.serve_tight_rtol > 0 and not args.serve_saturation_only and {"batched_f32", "one_at_a_time_f64"} <= set(forms):
        # the same two forms on the first requests of the stream solved to a tight tolerance, so that
        # FGMRES(30) runs deep Arnoldi cycles (and restarts) and the FP32 preconditioner is compared
        # with the FP64 one at an equal final residual on harder solves
        sub = reqs[:args.serve_tight_requests]
        tcommon = dict(common, rtol=args.serve_tight_rtol, maxit=3000)
        tforms = {"batched_f32": L.serve_config(prec="f32", max_active=args.serve_slots, **tcommon),
                  "one_at_a_time_f64": L.serve_config(prec="f64", max_active=1, **tcommon)}
        tight = {"rtol": args.serve_tight_rtol, "requests": len(sub)}
        for name, cfg in tforms.items():
            srv = L.Server(cfg, pool)
            res, el = srv.run(sub)
            stats = srv.stats()
            srv.destroy()
            lat = [r["t_done"] - r["t_arrival"] for r in res]
            tight[name] = {"solves_per_s": round(len(sub) / el, 2), "elapsed_s": round(el, 3), **percentiles(lat),
                           "converged": sum(1 for r in res if r["converged"] and r["rel_true_residual"] <= args.serve_tight_rtol),
                           "max_rel_true_residual": max(r["rel_true_residual"] for r in res),
                           "mean_iters": round(float(np.mean([r["iters"] for r in res])), 2),
                           "max_iters": int(max(r["iters"] for r in res)),
                           "solve_path_GBps": round(stats["bytes"] / el / 1e9, 1)}
            log(f"serving tight {name}: {tight[name]}")
        tight["speedup_solves_per_s"] = round(tight["batched_f32"]["solves_per_s"] /
                                              tight["one_at_a_time_f64"]["solves_per_s"], 3)
    cells = [L.abilu_gen_sizes(r)[0] for r in reqs]
    del pool
    torch.cuda.empty_cache()
    return {
        "workload": f"{len(reqs)} independent FGMRES(30) solves to rtol {args.rtol}: split-quad triangle or "
                    "anisotropic-quad meshes (50/50), cells log-uniform in [1e4, 1e6] "
                    f"(mean {np.mean(cells):.0f}, total {np.sum(cells)}), CFL ~ U(10, 1000), generated on the device",
        "preconditioner": f"ASYNC, {args.build_sweeps} factor sweep(s), {args.apply_sweeps} apply sweep pairs",
        "pool_GiB": args.serve_pool_gib, "slots": args.serve_slots,
        "saturation": sat,
        "kernel_profile_batched_f32": kernel_profile,
        "poisson": {"rate_per_s": round(lam, 2), **poisson} if lam else None,
        "poisson_high_load": poisson_high,
        "speedup_solves_per_s": (round(sat["batched_f32"]["solves_per_s"] / sat["one_at_a_time_f64"]["solves_per_s"], 3)
                                 if "batched_f32" in sat and "one_at_a_time_f64" in sat else None),
        "speedup_from_batching_f32": (round(sat["batched_f32"]["solves_per_s"] / sat["one_at_a_time_f32"]["solves_per_s"], 3)
                                      if "batched_f32" in sat and "one_at_a_time_f32" in sat else None),
        "tight_tolerance": tight,
    }


def warm_start_bench(args):
    """A pseudo-time sequence of drifting Jacobians on the 180,000-triangle mesh (CFL ramp 10 ->
    865 over 12 steps, 1% drift per step): one asynchronous FP32 factor sweep per step, from A
    (cold) or from the previous step's factor (warm), then FGMRES(30) to rtol."""
    import numpy as np
    import torch
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    c = W.case("tri300", cfl=10.0)
    cfls = W.cfl_ramp(args.warm_steps, 10.0, 1.5, 1000.0)
    sysm = {"cold": DeviceSystem(c, prec="f32", restart=30), "warm": DeviceSystem(c, prec="f32", restart=30)}
    rows = []
    for t, (vals, b) in enumerate(W.jacobian_sequence(c, cfls, drift=0.01, seed=args.serve_seed)):
        row = {"step": t, "cfl": round(float(cfls[t]), 2)}
        for name, s in sysm.items():
            s.load_values(vals, b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.factor(args.build_sweeps, "async", init="LU" if (name == "warm" and t > 0) else "A")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, res = s.solve(apply_sweeps=args.apply_sweeps, mode="async", rtol=args.rtol, maxit=300)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            row[name] = {"ilu_residual": float(f"{s.ilu_residual():.4e}"), "iters": res["iters"],
                         "converged": res["converged"], "factor_ms": round((t1 - t0) * 1e3, 3),
                         "solve_ms": round((t2 - t1) * 1e3, 3)}
        rows.append(row)
    log("warm start:", rows)
    tot = {k: {"iters": sum(r[k]["iters"] for r in rows),
               "mean_ilu_residual": float(np.mean([r[k]["ilu_residual"] for r in rows[1:]])) if len(rows) > 1 else None,
               "factor_ms": round(sum(r[k]["factor_ms"] for r in rows), 3),
               "solve_ms": round(sum(r[k]["solve_ms"] for r in rows), 3),
               "all_converged": all(r[k]["converged"] for r in rows)} for k in ("cold", "warm")}
    del sysm
    torch.cuda.empty_cache()
    out = {"workload": f"{c.n}-cell split-quad triangles, {len(rows)} pseudo-time steps, CFL {cfls[0]:g} -> "
                       f"{cfls[-1]:g}, 1% off-diagonal drift per step; async FP32, {args.build_sweeps} build sweep(s), "
                       f"{args.apply_sweeps} apply sweep pairs, FGMRES(30) to {args.rtol}",
           "totals": tot, "steps": rows}
    out["aniso1000_line_chunked"] = None if args.warm_steps_line <= 0 else warm_chunked_line(args)
    return out


def warm_chunked_line(args):
    """The same kind of sequence on the 500,000-cell boundary-layer mesh in line order: unchunked
    asynchronous sweeps from A, against chunked asynchronous sweeps (16-row chunks) from A (cold)
    and from the previous step's factor (warm). One FP32 factor sweep per step, FGMRES(30)."""
    import numpy as np
    import torch
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    c = W.case("aniso1000", order="line")
    cfls = W.cfl_ramp(args.warm_steps_line, 10.0, 1.5, 1000.0)
    forms = {"async_cold": ("async", "A"), "chunk_cold": ("chunk_async", "A"), "chunk_warm": ("chunk_async", "LU")}
    sysm = {k: DeviceSystem(c, prec="f32", restart=30) for k in forms}
    for k, (mode, _) in forms.items():
        if mode == "chunk_async":
            sysm[k].set_chunks(16)
    rows = []
    for t, (vals, b) in enumerate(W.jacobian_sequence(c, cfls, drift=0.01, seed=args.serve_seed)):
        row = {"step": t, "cfl": round(float(cfls[t]), 2)}
        for k, (mode, init) in forms.items():
            s = sysm[k]
            s.load_values(vals, b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.factor(args.build_sweeps, mode, init=init if t > 0 else "A")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, res = s.solve(apply_sweeps=args.apply_sweeps, mode=mode, rtol=args.rtol, maxit=300)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            row[k] = {"ilu_residual": float(f"{s.ilu_residual():.4e}"), "iters": res["iters"],
                      "converged": res["converged"], "factor_ms": round((t1 - t0) * 1e3, 3),
                      "solve_ms": round((t2 - t1) * 1e3, 3)}
        rows.append(row)
    log("warm start, line-ordered boundary layer:", rows)
    tot = {k: {"iters": sum(r[k]["iters"] for r in rows),
               "mean_ilu_residual": float(np.mean([r[k]["ilu_residual"] for r in rows[1:]])) if len(rows) > 1 else None,
               "factor_ms": round(sum(r[k]["factor_ms"] for r in rows), 3),
               "solve_ms": round(sum(r[k]["solve_ms"] for r in rows), 3),
               "all_converged": all(r[k]["converged"] for r in rows)} for k in forms}
    del sysm
    torch.cuda.empty_cache()
    return {"workload": f"{c.n}-cell boundary-layer quads in line order, {len(rows)} pseudo-time steps, CFL "
                        f"{cfls[0]:g} -> {cfls[-1]:g}, 1% drift per step; FP32, {args.build_sweeps} build sweep(s), "
                        f"{args.apply_sweeps} apply sweep pairs, FGMRES(30) to {args.rtol}",
            "totals": tot, "steps": rows}


def precision_bench(case, args):
    """The precision boundary: the headline step with the preconditioner in FP64 (factor storage and
    sweep arithmetic) beside FP32, the Krylov solver being FP64 in both; and, per workload, the error
    of the FP32 factor and application against the FP64 ones (precision_errors)."""
    import torch
    from paper_1912_00539_amd.runtime import DeviceSystem
    steps = {}
    for prec in ("f32", "f64"):
        s = DeviceSystem(case, prec=prec, restart=args.restart)
        run_steps(s, args, args.mode, 1, profile=False)
        nst = 3
        secs, res, rep = run_steps(s, args, args.mode, nst, profile=True)
        secs_np, res_np, _ = run_steps(s, args, args.mode, nst, profile=False)
        same = [r["iters"] for _, r in res_np] == [r["iters"] for _, r in res]
        t = secs_np if same else secs
        by = sum(v[2] for k, v in rep.items() if not k.startswith("_"))
        pre = {k: v for k, v in rep.items() if k.startswith(("factor_", "apply_"))}
        steps[prec] = {"ms_per_step": round(t * 1e3 / nst, 3), "GBps": round(by / t / 1e9, 1),
                       "preconditioner_bytes_per_step": round(sum(v[2] for v in pre.values()) / nst),
                       "preconditioner_ms_per_step": round(sum(v[1] for v in pre.values()) / nst, 3),
                       "fgmres_iters": [r["iters"] for _, r in res],
                       "max_rel_true_residual": max(r["rel_true_residual"] for _, r in res),
                       "ilu_residual": float(f"{s.ilu_residual():.4e}")}
        log(f"precision {prec}: {steps[prec]['ms_per_step']} ms/step, iters {steps[prec]['fgmres_iters']}")
        del s
        torch.cuda.empty_cache()
    f32, f64 = steps["f32"], steps["f64"]
    return {"mode": args.mode, "build_sweeps": args.build_sweeps, "apply_sweeps": args.apply_sweeps,
            "steps": steps,
            "f32_speedup_step": round(f64["ms_per_step"] / f32["ms_per_step"], 3),
            "f32_speedup_preconditioner": round(f64["preconditioner_ms_per_step"] / f32["preconditioner_ms_per_step"], 3),
            "f32_vs_f64": precision_errors(args)}


def _errors(a32, a64, bs):
    """Relative Frobenius error of a32 against a64, and the largest per-block relative error
    ||block difference||_F / ||block of a64||_F (blocks of `bs` consecutive values)."""
    d = a32.double() - a64
    nb = a64.numel() // bs
    dn = d[: nb * bs].reshape(nb, bs).norm(dim=1)
    an = a64[: nb * bs].reshape(nb, bs).norm(dim=1)
    nz = an > 0
    blk = (dn[nz] / an[nz]).max().item() if bool(nz.any()) else 0.0
    return {"rel": float(f"{(d.norm() / a64.norm()).item():.3e}"), "max_block_rel": float(f"{blk:.3e}")}


def precision_errors(args):
    """FP32 against FP64 on each full-size workload: the factor (X and Dinv) after 1 and 2
    synchronous sweeps, and one synchronous application (apply-sweeps pairs) of the 2-sweep factor
    to a seeded vector. The FP64 synchronous factor and application equal the FP64 oracle's bit for
    bit (the parity tests assert it), so these are the errors against the oracle."""
    import torch
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    out = {}
    for label, name, kw in (("tri300_cfl100", "tri300", {"cfl": 100.0}), ("aniso1000_line", "aniso1000", {"order": "line"}),
                            ("aniso1000_rcm", "aniso1000", {"order": "rcm"}), (args.workload, args.workload, {})):
        c = W.case(name, **kw)
        s = {p: DeviceSystem(c, prec=p, restart=1) for p in ("f32", "f64")}
        g = torch.Generator(device="cpu").manual_seed(args.serve_seed)
        r = (2 * torch.rand(4 * c.n, dtype=torch.float64, generator=g) - 1).cuda()
        row = {}
        for nsw in (1, 2):
            for p in s.values():
                p.factor(nsw, "sync")
            row[f"sweeps{nsw}"] = {"X": _errors(s["f32"].LU, s["f64"].LU, 16),
                                   "Dinv": _errors(s["f32"].Dinv, s["f64"].Dinv, 16)}
        z = {p: torch.zeros_like(r) for p in s}
        for p in s:
            s[p].apply(r, z[p], args.apply_sweeps, "sync")
        row["apply"] = _errors(z["f32"], z["f64"], 4)
        out[label] = row
        log(f"precision errors {label}: {row}")
        del s, z
        torch.cuda.empty_cache()
    return out


def configs_bench(args):
    """Factor and apply bandwidth on the other full-size workloads: one factor (init + 1 sweep) and
    one application (3 sweep pairs), SYNC and ASYNC, FP32 and FP64. The 180,000-triangle case fits
    the 256 MB Infinity Cache in part, so its figures are effective bandwidth, not HBM bandwidth."""
    import torch
    from paper_1912_00539_amd import abilu as L
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    out = {}
    for label, name, kw in (("tri300_cfl100", "tri300", {"cfl": 100.0}), ("aniso1000_line", "aniso1000", {"order": "line"}),
                            ("aniso1000_rcm", "aniso1000", {"order": "rcm"})):
        c = W.case(name, **kw)
        rows = {"n": c.n, "nnzb": c.nnzb}
        for prec in ("f32", "f64"):
            s = DeviceSystem(c, prec=prec, restart=1)
            r = torch.rand(4 * c.n, dtype=torch.float64, device="cuda")
            z = torch.zeros_like(r)
            for mode in ("sync", "async"):
                s.factor(1, mode)
                s.apply(r, z, args.apply_sweeps, mode)
                torch.cuda.synchronize()
                L.abilu_profile_enable(True, 100000)
                reps = 10
                for _ in range(reps):
                    s.factor(1, mode)
                    s.apply(r, z, args.apply_sweeps, mode)
                torch.cuda.synchronize()
                rep = L.abilu_profile_report()
                L.abilu_profile_enable(False)
                k = {kk: v for kk, v in rep.items() if kk.startswith(("factor_", "apply_"))}
                fb = sum(v[2] for kk, v in k.items() if kk.startswith("factor_"))
                fm = sum(v[1] for kk, v in k.items() if kk.startswith("factor_"))
                ab = sum(v[2] for kk, v in k.items() if kk.startswith("apply_"))
                am = sum(v[1] for kk, v in k.items() if kk.startswith("apply_"))
                rows[f"{prec}_{mode}"] = {
                    "factor_apply_GBps": round((fb + ab) / ((fm + am) / 1e3) / 1e9, 1),
                    "factor_ms": round(fm / reps, 4), "factor_GBps": round(fb / (fm / 1e3) / 1e9, 1),
                    "apply_ms": round(am / reps, 4), "apply_GBps": round(ab / (am / 1e3) / 1e9, 1),
                    "ilu_residual_1_sweep": float(f"{s.ilu_residual():.4e}")}
            del s
            torch.cuda.empty_cache()
        rows["working_set_note"] = ("partly cache-resident (effective bandwidth)" if c.n < 300000
                                    else "exceeds the 256 MB Infinity Cache")
        log(f"config {label}: {rows}")
        out[label] = rows
    out["quad32"] = config0_bench(args)
    out["tri300_cfl_sweep"] = tri300_sweep_bench()
    return out


def config0_bench(args):
    """The plain FP64 32x32 grid (1,024 cells) as specified: 3 synchronous factor sweeps, then one
    FGMRES(30) solve to 1e-2 with 3 synchronous apply sweep pairs, from a zero initial guess. A
    launch-bound workload: the time per factor and per solve (means over 200 repetitions) and the
    solve's iterations."""
    import torch
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    c = W.case("quad32")
    s = DeviceSystem(c, prec="f64", restart=30)
    s.factor(3, "sync")
    st, res = s.solve(apply_sweeps=3, mode="sync", rtol=1e-2, maxit=300)
    torch.cuda.synchronize()
    reps = 200
    t0 = time.perf_counter()
    for _ in range(reps):
        s.factor(3, "sync")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        st, res = s.solve(apply_sweeps=3, mode="sync", rtol=1e-2, maxit=300)
    t2 = time.perf_counter()
    out = {"n": c.n, "nnzb": c.nnzb, "factor_us": round((t1 - t0) / reps * 1e6, 1),
           "solve_us": round((t2 - t1) / reps * 1e6, 1), "fgmres_iters": res["iters"],
           "rel_true_residual": float(f"{res['rel_true_residual']:.4e}"), "converged": bool(res["converged"])}
    log(f"config 0 (quad32): {out}")
    del s
    torch.cuda.empty_cache()
    return out


def graphs_bench(args):
    """Launch overhead of small systems: a factor plus one application, issued as eager library
    calls and as one captured HIP graph replayed (the entry points launch kernels only, so they
    capture as they are). The plain FP64 32x32 grid (1,024 cells; 3 SYNC factor sweeps, 3 apply
    sweep pairs) and the 180,000-triangle mesh (FP32, 1 SYNC sweep, 3 pairs); the replayed factor
    and z are checked equal to the eager ones bit for bit."""
    import torch
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    out = {}
    for label, c, prec, nf in (("quad32_f64", W.case("quad32"), "f64", 3),
                               ("tri300_f32", W.case("tri300", cfl=100.0), "f32", 1)):
        s = DeviceSystem(c, prec=prec, restart=1)
        g_ = torch.Generator(device="cpu").manual_seed(args.serve_seed)
        r = (2 * torch.rand(4 * c.n, dtype=torch.float64, generator=g_) - 1).cuda()
        z = torch.zeros_like(r)

        def work():
            s.factor(nf, "sync")
            s.apply(r, z, args.apply_sweeps, "sync")

        work()
        torch.cuda.synchronize()
        X0, z0 = s.LU.clone(), z.clone()
        reps = 200
        t0 = time.perf_counter()
        for _ in range(reps):
            work()
        torch.cuda.synchronize()
        eager = (time.perf_counter() - t0) / reps
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            work()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            work()
        s.LU.fill_(float("nan"))
        z.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        same = bool(torch.equal(s.LU, X0) and torch.equal(z, z0))
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        graph = (time.perf_counter() - t0) / reps
        out[label] = {"n": c.n, "factor_sweeps": nf, "apply_sweeps": args.apply_sweeps,
                      "eager_us": round(eager * 1e6, 1), "graph_us": round(graph * 1e6, 1),
                      "speedup": round(eager / graph, 2), "replay_bits_equal": same}
        log(f"graphs {label}: {out[label]}")
        del g, s
        torch.cuda.empty_cache()
    return out


def tri300_sweep_bench():
    """The 180,000-triangle workload at CFL 10, 100 and 1000: ILU residual after 1 to 4 FP32 factor
    sweeps, SYNC and ASYNC, and the FGMRES(30) iterations to 1e-2 with 2 apply sweep pairs."""
    import torch
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    out = {}
    for cfl in (10.0, 100.0, 1000.0):
        c = W.case("tri300", cfl=cfl)
        s = DeviceSystem(c, prec="f32", restart=30)
        rows = []
        for nsw in (1, 2, 3, 4):
            row = {"factor_sweeps": nsw}
            for mode in ("sync", "async"):
                s.factor(nsw, mode)
                ilu = s.ilu_residual()
                st, res = s.solve(apply_sweeps=2, mode=mode, rtol=1e-2, maxit=300)
                row[mode] = {"ilu_residual": float(f"{ilu:.4e}"), "fgmres_iters": res["iters"],
                             "converged": bool(res["converged"])}
            rows.append(row)
        log(f"tri300 CFL {cfl:g}: {rows}")
        out[f"cfl{cfl:g}"] = rows
        del s
        torch.cuda.empty_cache()
    return out


def factor_convergence_bench(args):
    """The ILU-convergence study of Section 6.2 on the full-size workloads: the factor errors
    ||vec(L - L_ilu)||_inf / ||vec(L0 - L_ilu)||_inf and likewise for U, and the ILU residual,
    after 1 to 5 factor sweeps from A, for SYNC, ASYNC and CHUNK_ASYNC in FP64 and FP32; the
    asynchronous modes run 5 times (mean, min, max), as the paper averages 5 runs; and the Jacobi
    max-norms of the final factors and of X_ilu. X_ilu is the floating-point fixed point of the FP64
    synchronous sweeps, reached by sweeping until an iterate repeats bit for bit: the map is
    triangular in the Gaussian-elimination ordering, so that fixed point is unique and is the
    sequential block ILU(0) (the GPU tests check this against the oracle)."""
    import numpy as np
    import torch
    from paper_1912_00539_amd import abilu as L
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    out, summary = {}, {}
    nsws = list(range(1, 6))
    for label, name, kw, R in (("aniso1000_line", "aniso1000", {"order": "line"}, 16),
                               (args.workload, args.workload, {}, 64)):
        c = W.case(name, **kw)
        ref = DeviceSystem(c, prec="f64", restart=0)
        ref.factor(1, "sync")
        prev = ref.LU.clone()
        fixed = None
        for q in range(2, args.fixed_point_cap + 1):
            ref.factor(1, "sync", init="LU")
            if torch.equal(ref.LU, prev):
                fixed = q - 1
                break
            prev.copy_(ref.LU)
        del prev
        Y, DY = ref.LU, ref.Dinv
        X0 = torch.empty_like(Y)
        L.abilu_factor_from_csr(ref.pattern, "f64", ref.A, X0)
        dL, dU = L.abilu_factor_maxdiff(ref.pattern, "f64", X0, Y, ref.work)
        del X0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D, nl, nu = L.abilu_pattern_depth(ref.pattern)
        t_depth = time.perf_counter() - t0
        row = {"n": c.n, "nnzb": c.nnzb, "depth_D": D, "levels_lower": nl, "levels_upper": nu,
               "depth_analysis_ms": round(t_depth * 1e3, 1), "sweeps_to_fixed_point": fixed,
               "x_ilu_ilu_residual": float(f"{ref.ilu_residual():.3e}"),
               "x_ilu_jacobi_norms": [float(f"{v:.4g}") for v in L.abilu_jacobi_norms(ref.pattern, "f64", Y, DY, ref.work)],
               "initial_maxdiff": [dL, dU], "runs": {}}
        log(f"factor convergence {label}: X_ilu after {fixed} sweeps")
        for prec in ("f64", "f32"):
            for mode, reps in (("sync", 1), ("async", 5), ("chunk_async", 5)):
                s = DeviceSystem(c, prec=prec, restart=0)
                if mode == "chunk_async":
                    s.set_chunks(R)
                eL = np.zeros((reps, len(nsws)))
                eU = np.zeros_like(eL)
                ilu = np.zeros_like(eL)
                for t in range(reps):
                    for k, nsw in enumerate(nsws):
                        s.factor(nsw, mode)
                        nL, nU = L.abilu_factor_maxdiff(s.pattern, prec, s.LU, Y, s.work)
                        eL[t, k] = nL / dL if dL > 0 else nL
                        eU[t, k] = nU / dU if dU > 0 else nU
                        ilu[t, k] = s.ilu_residual()
                jn = L.abilu_jacobi_norms(s.pattern, prec, s.LU, s.Dinv, s.work)
                f = lambda a: [float(f"{v:.3e}") for v in a]
                r = {"E_L_mean": f(eL.mean(0)), "E_U_mean": f(eU.mean(0)), "ilu_residual_mean": f(ilu.mean(0)),
                     "jacobi_norms_final": [float(f"{v:.4g}") for v in jn], "runs": reps}
                if reps > 1:
                    r.update({"E_L_min": f(eL.min(0)), "E_L_max": f(eL.max(0)), "E_U_min": f(eU.min(0)),
                              "E_U_max": f(eU.max(0)), "ilu_residual_min": f(ilu.min(0)),
                              "ilu_residual_max": f(ilu.max(0))})
                row["runs"][f"{prec}_{mode}"] = r
                log(f"factor convergence {label} {prec} {mode}: {r}")
                del s
                torch.cuda.empty_cache()
        out[label] = row
        a = row["runs"]["f32_async"]
        summary[label] = {"D": D, "fixed_point_sweeps": fixed, "f32_async_E_L": a["E_L_mean"],
                          "f32_async_E_U": a["E_U_mean"]}
        del ref, Y, DY
        torch.cuda.empty_cache()
    out["sweeps"] = nsws
    out["summary"] = summary
    return out


def orderings_bench(args):
    """Orderings of mesh cells (Section 5) computed by the library (host), the same seeded matrix
    assembled in each, then the step (FP32 preconditioner, 1 build sweep, 3 apply sweep pairs,
    FGMRES to rtol) with unchunked asynchronous sweeps and with chunked ones (Gauss-Seidel within
    chunks of consecutive rows, where the ordering decides which dependencies fall inside a chunk):
    on the 500,000-cell boundary-layer mesh (lines found from the geometric face couplings,
    anisotropy threshold 10, strong-link ratio 4; 16-row chunks) and on the 180,000-triangle mesh
    from a random numbering (RCM, 1WD; 64-row chunks)."""
    import numpy as np
    import torch
    from paper_1912_00539_amd import abilu as L
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    out = {}
    studies = (("aniso1000", W.aniso_quad_mesh(1000, 500), "natural", 100.0,
                ("line_columns", "rcm", "1wd", "line", "line_rcm", "line_1wd"), 16),
               ("tri300", W.split_tri_mesh(300, 300, args.serve_seed), "random", 100.0, ("random", "rcm", "1wd"), 64))
    for label, m, start, cfl, names, R in studies:
        seed = args.serve_seed
        if start == "natural":
            base = W.natural_order(m)
        else:
            base = np.argsort(np.argsort(W.uniform01(seed, W.S_PERM, np.arange(m.ncells)), kind="stable"),
                              kind="stable")
        c0 = W.assemble(m, base, seed, "cfl", cfl=cfl)
        wgt = W.block_face_weights(m, base, c0.rowptr, c0.colidx)
        t = time.perf_counter()
        lo, lp, nl = L.abilu_find_lines(c0.n, c0.rowptr, c0.colidx, wgt, 10.0, 4.0)
        t_lines = time.perf_counter() - t
        rows = {"n": c0.n, "lines": nl, "cells_in_lines": int((lo >= 0).sum()),
                "find_lines_ms": round(t_lines * 1e3, 1), "rows_per_chunk": R}
        for name in names:
            t = time.perf_counter()
            if name == "line_columns":
                new = W.line_order(m)                       # whole wall-normal columns (generator)
            elif name == "random":
                new = np.arange(m.ncells)
            else:
                new_c = L.abilu_order(c0.n, c0.rowptr, c0.colidx, name, lo, lp).astype(np.int64)
                new = new_c[base]                           # compose: natural -> base -> new
            t_ord = time.perf_counter() - t
            c = W.assemble(m, new if name != "random" else base, seed, "cfl", cfl=cfl)
            s = DeviceSystem(c, prec="f32", restart=args.restart)
            rows[name] = {"ordering_ms": None if name in ("line_columns", "random") else round(t_ord * 1e3, 1)}
            for mode in ("async", "chunk_async"):
                if mode == "chunk_async":
                    rows[name]["chunk_runner"] = s.set_chunks(R)["runner"]
                run_steps(s, args, mode, 1, profile=False)
                nst = 3
                secs, res = run_steps(s, args, mode, nst, profile=False)[:2]
                rows[name][mode] = {"ilu_residual": float(f"{s.ilu_residual():.4e}"),
                                    "fgmres_iters": [r["iters"] for _, r in res],
                                    "max_rel_true_residual": max(r["rel_true_residual"] for _, r in res),
                                    "ms_per_step": round(secs * 1e3 / nst, 3)}
            log(f"ordering {label} {name}: {rows[name]}")
            del s
            torch.cuda.empty_cache()
        out[label] = rows
    return out


def chunked_bench(args):
    """Chunked sweeps (Gauss-Seidel within chunks of consecutive rows, the schedule of the paper's
    OpenMP chunks) against the unchunked asynchronous sweeps, same step otherwise (FP32
    preconditioner, 1 build sweep, 3 apply sweep pairs, FGMRES to rtol), on the headline 4M-cell
    triangles (64-row chunks) and on the 500,000-cell anisotropic quads in line order, where each
    chunk is a run of one wall-normal line (16-row chunks)."""
    import torch
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem
    out = {}
    for label, name, kw, R in (("tri2000", args.workload, {}, 64),
                               ("aniso1000_line", "aniso1000", {"order": "line"}, 16)):
        c = W.case(name, **kw)
        s = DeviceSystem(c, prec=args.prec, restart=args.restart)
        rows = {}
        for mode in ("async", "chunk_async"):
            info = s.set_chunks(R) if mode == "chunk_async" else None
            run_steps(s, args, mode, 1, profile=False)
            nst = 5
            secs, res, rep = run_steps(s, args, mode, nst, profile=True)
            secs_np, res_np, _ = run_steps(s, args, mode, nst, profile=False)
            same = [r["iters"] for _, r in res_np] == [r["iters"] for _, r in res]
            t = secs_np if same else secs
            by = sum(v[2] for k, v in rep.items() if not k.startswith("_"))
            fs = {k: v for k, v in rep.items() if k.startswith("factor_sweep")}
            ap = {k: v for k, v in rep.items() if k.startswith("apply_")}
            rows[mode] = {"ms_per_step": round(t * 1e3 / nst, 3), "GBps": round(by / t / 1e9, 1),
                          "fgmres_iters": [r["iters"] for _, r in res],
                          "max_rel_true_residual": max(r["rel_true_residual"] for _, r in res),
                          "ilu_residual": float(f"{s.ilu_residual():.4e}"),
                          "factor_sweep_ms": round(sum(v[1] for v in fs.values()) / max(1, sum(v[0] for v in fs.values())), 4),
                          "factor_sweep_GBps": round(sum(v[2] for v in fs.values()) / (sum(v[1] for v in fs.values()) / 1e3) / 1e9, 1),
                          "apply_GBps": round(sum(v[2] for v in ap.values()) / (sum(v[1] for v in ap.values()) / 1e3) / 1e9, 1)}
            if info:
                rows[mode]["chunks"] = {k: info[k] for k in ("rows_per_chunk", "nchunks", "runner", "max_levels_lower",
                                                             "levels_lower")}
            log(f"chunked {label} {mode}: {rows[mode]}")
        rows["chunk_over_async_step_time"] = round(rows["chunk_async"]["ms_per_step"] / rows["async"]["ms_per_step"], 3)
        out[label] = {"n": c.n, "nnzb": c.nnzb, **rows}
        del s
        torch.cuda.empty_cache()
    return out


# Kernels of the headline step (rocprofv3's demangled names) and the names the library's profiler
# gives their launches in the asynchronous FP32 step.
TRAFFIC_KERNELS = {
    "k_spmv<false>": "spmv", "k_spmv<true>": "spmv_resid",
    "k_factor_sweep<float, false, true, true>": "factor_sweep_f32_async_fromA",
    "k_fwd<float, double, false>": "apply_fwd_f32_async", "k_fwd<float, float, true>": "apply_fwd_emitz_f32_async",
    "k_bwd<float, float, float, true, false>": "apply_bwd_f32_async",
    "k_bwd<float, float, double, true, false>": "apply_bwd_last_f32_async",
    "k_update": "fgmres_update", "k_mdot": "fgmres_mdot", "k_stream_copy": "stream_copy",
}


def kernel_short_name(name):
    """rocprofv3's kernel name without return type, namespace and parameter list: k_spmv<false>."""
    n = name.replace("(anonymous namespace)::", "").strip()
    if n.startswith("void "):
        n = n[5:]
    return n.split("(")[0].strip()


def _csv_rows(d, suffix):
    import csv
    import glob
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            out += list(csv.DictReader(fh))
    return out


def summarize_stats(d, title, command):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (its *kernel_stats.csv)."""
    rows = _csv_rows(d, "kernel_stats.csv")
    if not rows:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    for r in rows:
        r["Name"] = kernel_short_name(r["Name"])
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics: {title}", "", "Command (run from the repository root on an MI355X machine):",
             "", "```", command, "```", "", "| kernel | calls | avg us | min us | max us | total ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{100 * float(r['TotalDurationNs']) / tot:.2f} |")
    lines += ["", f"Total kernel time {tot / 1e6:.3f} ms."]
    return "\n".join(lines) + "\n"


def summarize_trace_segments(d, marker, title, command, seg_titles):
    """Markdown tables of a rocprofv3 --kernel-trace run (its *kernel_trace.csv) split into segments,
    each starting at a dispatch of the kernel `marker` (e.g. each workload's pattern build)."""
    rows = _csv_rows(d, "kernel_trace.csv")
    if not rows:
        raise SystemExit(f"no kernel_trace.csv under {d}")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    starts = [q for q, r in enumerate(rows) if kernel_short_name(r["Kernel_Name"]) == marker]
    if len(starts) != len(seg_titles):
        raise SystemExit(f"{len(starts)} segments start with {marker}, {len(seg_titles)} titles given")
    lines = [f"# rocprofv3 kernel statistics: {title}", "", "Command (run from the repository root on an MI355X machine):",
             "", "```", command, "```"]
    for q, st in enumerate(starts):
        seg = rows[st:starts[q + 1] if q + 1 < len(starts) else len(rows)]
        acc = {}
        for r in seg:
            name = kernel_short_name(r["Kernel_Name"])
            acc.setdefault(name, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        tot = sum(sum(v) for v in acc.values())
        lines += ["", f"## {seg_titles[q]}", "", "| kernel | calls | avg us | min us | max us | total ms | % |",
                  "|---|---:|---:|---:|---:|---:|---:|"]
        for name, v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
            if sum(v) < 0.001 * tot:
                continue
            lines.append(f"| `{name}` | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
                         f"{sum(v) / 1e3:.3f} | {100 * sum(v) / tot:.2f} |")
        lines += ["", f"Segment kernel time {tot / 1e3:.3f} ms (kernels under 0.1% of it left out)."]
    return "\n".join(lines) + "\n"


def summarize_traffic(fetch_dir, write_dir, command):
    """Bytes per launch of the headline step's kernels from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE, KiB per dispatch), each scaled by the ratio of the known bytes of the STREAM
    copy kernel (its reads, its writes) to what the counter reads for it. Returns (json, markdown)."""
    import numpy as np

    def per_kernel(d, counter):
        acc = {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            name = kernel_short_name(r["Kernel_Name"])
            acc.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0)
        return acc
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = STREAM_BYTES // 2      # bytes read (and written) by one STREAM copy launch
    cf = copy_bytes / float(np.median(fetch["k_stream_copy"]))
    cw = copy_bytes / float(np.median(write["k_stream_copy"]))
    shash = source_hash()
    out = {"_source": "rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (separate runs), KiB per dispatch, scaled by "
                      "the ratio of the known bytes of a 2 GiB STREAM copy to what each counter reads for it",
           "copy_factor_fetch": cf, "copy_factor_write": cw}
    md = ["# Measured L2-to-memory traffic per launch: tri2000 (4M cells), async FP32 step", "",
          "Command (run from the repository root on an MI355X machine):", "", "```", command, "```", "",
          f"Calibration: the 2 GiB STREAM copy reads {1 / cf:.3f}x its bytes in FETCH_SIZE and {1 / cw:.3f}x in "
          f"WRITE_SIZE; every figure below is scaled by those factors ({cf:.3f}, {cw:.3f}).", "",
          "| kernel (library name) | dispatches | fetch MB | write MB | total MB per launch |",
          "|---|---:|---:|---:|---:|"]
    for kname, lname in TRAFFIC_KERNELS.items():
        if kname not in fetch or kname not in write:
            continue
        f = float(np.median(fetch[kname])) * cf
        w = float(np.median(write[kname])) * cw
        out[lname] = {"dispatches": len(fetch[kname]), "fetch_bytes_per_launch": round(f),
                      "write_bytes_per_launch": round(w), "bytes_per_launch": round(f + w), "source_hash": shash}
        md.append(f"| `{lname}` | {len(fetch[kname])} | {f / 1e6:.1f} | {w / 1e6:.1f} | {(f + w) / 1e6:.1f} |")
    md += ["", f"Kernel source hash when measured: `{shash}` (bench.py reports this traffic only while the hash matches)."]
    return json.dumps(out, indent=1) + "\n", "\n".join(md) + "\n"


def summarize_serving_traffic(fetch_dir, write_dir, cf, cw, command):
    """Measured bytes of the serving run per kernel, summed over its dispatches, from two
    rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE), scaled by the STREAM-copy calibration
    factors cf, cw of the headline traffic measurement. Solve kernels (kb_*) and admission kernels
    (kbs_*) are totalled separately. Returns markdown."""
    def per_kernel(d, counter, f):
        acc = {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            name = kernel_short_name(r["Kernel_Name"])
            n, b = acc.get(name, (0, 0.0))
            acc[name] = (n + 1, b + float(r["Counter_Value"]) * 1024.0 * f)
        return acc
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE", cf), per_kernel(write_dir, "WRITE_SIZE", cw)
    names = sorted(set(fetch) | set(write), key=lambda k: -(fetch.get(k, (0, 0))[1] + write.get(k, (0, 0))[1]))
    md = ["# Measured HBM traffic of the serving run: 2000 requests released at t = 0, batched FP32 preconditioner",
          "", "Command (run from the repository root on an MI355X machine):", "", "```", command, "```", "",
          f"FETCH_SIZE and WRITE_SIZE (KiB per dispatch) summed over each kernel's dispatches and scaled by the "
          f"STREAM-copy calibration of the headline traffic measurement ({cf:.3f}, {cw:.3f}). `kb_*` are the "
          "batched solve kernels, `kbs_*` the admission kernels (matrix generation and pattern analysis of "
          "arriving requests), which run concurrently on a second stream.", "",
          "| kernel | dispatches | fetch GB | write GB | total GB |", "|---|---:|---:|---:|---:|"]
    groups = {"solve (kb_*)": 0.0, "admission (kbs_*)": 0.0, "other": 0.0}
    for k in names:
        n = max(fetch.get(k, (0, 0))[0], write.get(k, (0, 0))[0])
        f, w = fetch.get(k, (0, 0.0))[1], write.get(k, (0, 0.0))[1]
        g = "admission (kbs_*)" if k.startswith("kbs_") else ("solve (kb_*)" if k.startswith("kb_") else "other")
        groups[g] += f + w
        if f + w >= 1e9:
            md.append(f"| `{k}` | {n} | {f / 1e9:.2f} | {w / 1e9:.2f} | {(f + w) / 1e9:.2f} |")
    md += ["", "Kernels under 1 GB are left out of the table and counted in the totals.", "",
           "| group | total GB |", "|---|---:|"]
    for g, b in groups.items():
        md.append(f"| {g} | {b / 1e9:.1f} |")
    md.append(f"| all | {sum(groups.values()) / 1e9:.1f} |")
    return "\n".join(md) + "\n"


def summarize_launch_traffic(fetch_dir, write_dir, cf, cw, title, command):
    """Measured bytes per launch (medians over dispatches) of every kernel of a run, split by grid
    size (one run may cover several workloads), from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE), scaled by the STREAM-copy calibration factors cf, cw. Returns markdown."""
    import numpy as np

    def per_kernel(d, counter, f):
        acc = {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            key = (kernel_short_name(r["Kernel_Name"]), int(r.get("Grid_Size", 0) or 0))
            acc.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0 * f)
        return acc
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE", cf), per_kernel(write_dir, "WRITE_SIZE", cw)
    keys = sorted(set(fetch) & set(write), key=lambda k: (k[0], -k[1]))
    md = [f"# Measured L2-to-memory traffic per launch: {title}", "", "Command (run from the repository root on an MI355X "
          "machine):", "", "```", command, "```", "",
          f"Medians over each kernel's dispatches, split by grid size (threads), scaled by the STREAM-copy "
          f"calibration of the headline traffic measurement ({cf:.3f}, {cw:.3f}).", "",
          "| kernel | grid | dispatches | fetch MB | write MB | total MB per launch |", "|---|---:|---:|---:|---:|---:|"]
    for k in keys:
        f, w = float(np.median(fetch[k])), float(np.median(write[k]))
        if f + w < 1e6 or not k[0].startswith("k"):
            continue
        md.append(f"| `{k[0]}` | {k[1]} | {len(fetch[k])} | {f / 1e6:.1f} | {w / 1e6:.1f} | {(f + w) / 1e6:.1f} |")
    md += ["", "Library kernels only; launches under 1 MB are left out."]
    return "\n".join(md) + "\n"


STREAM_BYTES = 2 * (2 << 30)   # algorithmic bytes of one stream_reference copy launch (read + write)


def main():
    if len(sys.argv) > 1 and sys.argv[1] in ("--summarize-stats", "--summarize-traffic",
                                             "--summarize-serving-traffic", "--summarize-launch-traffic",
                                             "--summarize-trace-segments"):
        return summarize_main(sys.argv[1:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="async", choices=["sync", "async"])
    ap.add_argument("--compare", default="sync:1:100,sync:2:500",
                    help="comma list of mode:build_sweeps:maxit runs reported beside the headline ('none' to skip)")
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default="tri2000")
    ap.add_argument("--build-sweeps", type=int, default=1)
    ap.add_argument("--apply-sweeps", type=int, default=3)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--maxit", type=int, default=500)
    ap.add_argument("--rtol", type=float, default=1e-2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-seed", type=int, default=7)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-pool-gib", type=float, default=64.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-forms", default="batched_f32,one_at_a_time_f64,one_at_a_time_f32")
    ap.add_argument("--serve-saturation-only", action="store_true")
    ap.add_argument("--serve-tight-rtol", type=float, default=1e-8,
                    help="also solve the first --serve-tight-requests requests to this tolerance (0: skip)")
    ap.add_argument("--serve-tight-requests", type=int, default=400)
    ap.add_argument("--serve-profile", action="store_true",
                    help="add a profiled saturation run of the batched form (per-kernel GB/s)")
    ap.add_argument("--warm-steps", type=int, default=12)
    ap.add_argument("--warm-steps-line", type=int, default=8)
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-chunked", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--no-orderings", action="store_true")
    ap.add_argument("--no-factor-convergence", action="store_true")
    ap.add_argument("--fixed-point-cap", type=int, default=400,
                    help="most FP64 synchronous sweeps spent looking for the fixed point X_ilu")
    ap.add_argument("--only-factor-convergence", action="store_true",
                    help="print the factor_convergence object alone")
    ap.add_argument("--only-orderings", action="store_true", help="print the orderings object alone")
    ap.add_argument("--only-warm", action="store_true", help="print the warm_start object alone")
    ap.add_argument("--only-chunked", action="store_true", help="print the chunked object alone")
    ap.add_argument("--only-serving", action="store_true", help="print the serving object alone (profiling)")
    ap.add_argument("--detail", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file that receives the full result object (the last stdout line is the compact headline)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU (asked for {args.gpus} GPUs, WORLD_SIZE={world}); "
              "a multi-GPU decomposition is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_00539_amd import abilu as L
    from paper_1912_00539_amd import workloads as W
    from paper_1912_00539_amd.runtime import DeviceSystem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    L.lib()
    if args.only_serving:
        print(json.dumps({"serving": serving_bench(args)}), flush=True)
        return
    if args.only_warm:
        print(json.dumps({"warm_start": warm_start_bench(args)}), flush=True)
        return
    if args.only_orderings:
        print(json.dumps({"orderings": orderings_bench(args)}), flush=True)
        return
    if args.only_factor_convergence:
        print(json.dumps({"factor_convergence": factor_convergence_bench(args)}), flush=True)
        return
    if args.only_chunked:
        print(json.dumps({"chunked": chunked_bench(args)}), flush=True)
        return
    t = time.perf_counter()
    case = W.case(args.workload)
    log(f"generated {args.workload}: N={case.n} Z={case.nnzb} in {time.perf_counter() - t:.1f} s")
    sysm = DeviceSystem(case, prec=args.prec, restart=args.restart)
    n, z, npairs = sysm.pattern.info()
    log(f"pattern built: npairs={npairs}; workspace {sysm.work.numel() / 2**30:.2f} GiB")

    stream_gbps = None if args.no_stream else stream_reference()
    if stream_gbps:
        log(f"STREAM copy reference: {stream_gbps:.0f} GB/s")

    run_steps(sysm, args, args.mode, args.warmup, profile=False)
    log(f"warmup done ({args.warmup} steps)")
    secs, results, rep = run_steps(sysm, args, args.mode, args.steps, profile=True)
    log(f"timed {args.steps} steps: {secs * 1e3 / args.steps:.3f} ms/step")
    secs_np, results_np, _ = run_steps(sysm, args, args.mode, args.steps, profile=False)
    log(f"timed {args.steps} steps without profiling: {secs_np * 1e3 / args.steps:.3f} ms/step")
    # The profiled run records a HIP event pair around every launch; the whole-job rate is taken
    # from the run without them, whose work is the same launch sequence (checked: identical
    # FGMRES iteration counts, hence identical algorithmic bytes).
    same_work = [r["iters"] for _, r in results_np] == [r["iters"] for _, r in results]
    secs_value = secs_np if same_work else secs
    ilu_res = sysm.ilu_residual()

    kernels = {k: v for k, v in rep.items() if not k.startswith("_")}
    total_bytes = sum(v[2] for v in kernels.values())
    total_kernel_ms = sum(v[1] for v in kernels.values())
    value = total_bytes / secs_value / 1e9
    fa = {k: v for k, v in kernels.items() if k.startswith(("factor_", "apply_"))}
    fa_bytes = sum(v[2] for v in fa.values())
    fa_ms = sum(v[1] for v in fa.values())
    sweeps = sum(v[0] for k, v in kernels.items() if k.startswith("factor_sweep"))
    sweep_ms = sum(v[1] for k, v in kernels.items() if k.startswith("factor_sweep"))
    dom = max(kernels.items(), key=lambda kv: kv[1][1])
    dname, (dcnt, dms, dbytes) = dom
    achieved = dbytes / (dms / 1e3) / 1e9
    shash = source_hash()
    traffic = load_traffic(dname, shash)
    iters = [r["iters"] for _, r in results]
    conv = all(r["converged"] for _, r in results)
    resid = max(r["rel_true_residual"] for _, r in results)

    compare = []
    if args.compare != "none":
        for spec in args.compare.split(","):
            cmode, cnb, cmaxit = spec.split(":")
            cnb, cmaxit = int(cnb), int(cmaxit)
            run_steps(sysm, args, cmode, 1, profile=False, build_sweeps=cnb, maxit=cmaxit)
            nst = 3
            csecs, cres, crep = run_steps(sysm, args, cmode, nst, profile=True, build_sweeps=cnb, maxit=cmaxit)
            cb = sum(v[2] for k, v in crep.items() if not k.startswith("_"))
            compare.append({"mode": cmode, "build_sweeps": cnb, "maxit": cmaxit,
                            "ms_per_step": round(csecs * 1e3 / nst, 3), "GBps": round(cb / csecs / 1e9, 1),
                            "fgmres_iters": [r["iters"] for _, r in cres],
                            "converged": all(r["converged"] for _, r in cres),
                            "ilu_residual": sysm.ilu_residual()})
        log("compare:", compare)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs_value * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.prec == "f32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: 2000x1000 quads split into {case.n} triangles, {case.nnzb} 4x4 blocks, "
                        "CFL 100, random permutation + RCM",
            "mode": args.mode, "build_sweeps": args.build_sweeps, "apply_sweeps": args.apply_sweeps,
            "fgmres_restart": args.restart, "rtol": args.rtol, "factor_precision": args.prec,
            "krylov_precision": "f64"},
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "launches": dcnt, "avg_launch_ms": round(dms / dcnt, 5),
                     "algorithmic_bytes_per_launch": round(dbytes / dcnt)},
        "frac_hbm_peak": round(value / HBM_PEAK_GBPS, 4),
        "stream_copy_GBps": round(stream_gbps, 1) if stream_gbps else None,
        "frac_stream": round(value / stream_gbps, 4) if stream_gbps else None,
        "factor_apply_GBps": round(fa_bytes / (fa_ms / 1e3) / 1e9, 1) if fa_ms else None,
        "factor_sweeps_per_s": round(sweeps / (sweep_ms / 1e3), 1) if sweep_ms else None,
        "solves_per_s": round(args.steps / secs_value, 3),
        "timing": "without per-launch profiling events" if same_work else
                  "profiled run (the unprofiled run did different work)",
        "ms_per_step_profiled": round(secs * 1e3 / args.steps, 3),
        "value_profiled_GBps": round(total_bytes / secs / 1e9, 1),
        "kernel_time_frac_of_profiled_step": round(total_kernel_ms / (secs * 1e3), 3),
        "fgmres_iters": iters,
        "ilu_residual": ilu_res,
        "converged": conv,
        "max_rel_true_residual": resid,
        "kernels": {k: {"launches": v[0], "ms": round(v[1], 4), "GBps": round(v[2] / (v[1] / 1e3) / 1e9, 1) if v[1] else None}
                    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1][1])},
        "compare": compare,
        "source_hash": shash,
    }
    del sysm
    torch.cuda.empty_cache()
    out["precision"] = None if args.no_precision else precision_bench(case, args)
    out["chunked"] = None if args.no_chunked else chunked_bench(args)
    out["configs"] = None if args.no_configs else configs_bench(args)
    out["graphs"] = None if args.no_graphs else graphs_bench(args)
    out["orderings"] = None if args.no_orderings else orderings_bench(args)
    out["serving"] = None if args.no_serving else serving_bench(args)
    out["warm_start"] = None if args.no_warm_start else warm_start_bench(args)
    out["factor_convergence"] = None if args.no_factor_convergence else factor_convergence_bench(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(case, args, gpu=gpu_sync_factors(case))
    else:
        out["cpu_baseline"] = None
    emit(out, args.detail)


def emit(out, detail_path):
    """Write the full result object to `detail_path` (and to stderr), then print the compact
    headline as the last line of stdout."""
    text = json.dumps(out)
    if detail_path:
        d = os.path.dirname(os.path.abspath(detail_path))
        os.makedirs(d, exist_ok=True)
        with open(detail_path, "w") as f:
            f.write(text + "\n")
    log("detail:", text)
    head = headline(out, detail_path)
    print(json.dumps(head, separators=(",", ":")), flush=True)


def _pick(d, *keys):
    return {k: d.get(k) for k in keys} if d else None


def _sig(x, n=4):
    """x with every float rounded to n significant digits (nested dicts and lists too)."""
    if isinstance(x, float):
        return float(f"{x:.{n - 1}e}") if x == x and abs(x) != float("inf") else x
    if isinstance(x, dict):
        return {k: _sig(v, n) for k, v in x.items()}
    if isinstance(x, list):
        return [_sig(v, n) for v in x]
    return x


def headline(out, detail_path=None):
    """The compact result line (a few KB): the headline figures of `out` and a summary of every
    sub-benchmark, the full object being in the detail file. Secondary figures (residuals, errors,
    serving and convergence summaries) are rounded to 4 significant digits; the detail file keeps
    them whole."""
    h = {k: out.get(k) for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                 "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config")}
    h["value_covers"] = "whole step (factor, FGMRES with apply sweeps, SpMV, Gram-Schmidt): algorithmic bytes / wall time"
    rl = out.get("roofline") or {}
    h["roofline"] = _pick(rl, "bound", "kernel", "achieved", "peak", "unit", "frac", "traffic", "avg_launch_ms",
                          "algorithmic_bytes_per_launch")
    for k in ("frac_hbm_peak", "stream_copy_GBps", "frac_stream", "factor_apply_GBps", "factor_sweeps_per_s",
              "solves_per_s", "converged", "max_rel_true_residual", "ilu_residual", "timing"):
        h[k] = out.get(k)
    if out.get("factor_apply_GBps"):
        h["factor_apply_frac_hbm_peak"] = round(out["factor_apply_GBps"] / HBM_PEAK_GBPS, 4)
    it = out.get("fgmres_iters") or []
    h["fgmres_iters"] = [min(it), max(it)] if it else None
    cpu = out.get("cpu_baseline")
    if cpu:
        h["cpu_baseline"] = {**_pick(cpu, "value", "unit", "cores", "kind", "cpu_model", "host_cpus", "seconds"),
                             "sample": cpu.get("sample"),
                             "sequential_ms": _pick(cpu.get("sequential") or {}, "ilu0_ms", "exact_substitution_ms"),
                             "oracle_check": {k: v for k, v in (cpu.get("oracle_check") or {}).items()
                                              if k != "what"} or None}
    else:
        h["cpu_baseline"] = None
    sv = out.get("serving")
    if sv:
        sat = sv.get("saturation") or {}
        po = sv.get("poisson") or {}
        form = lambda r, keys: _pick(r, *keys) if r else None
        h["serving"] = {
            "requests": (sat.get("batched_f32") or {}).get("converged"),
            "saturation": {k: form(sat.get(k), ("solves_per_s", "p50_ms", "p99_ms", "solve_path_GBps", "mean_iters",
                                                "max_rel_true_residual") if k != "one_at_a_time_f32"
                                   else ("solves_per_s",)) for k in sat},
            "speedup_solves_per_s": sv.get("speedup_solves_per_s"),
            "poisson_rate_per_s": po.get("rate_per_s"),
            "poisson": {k: form(po.get(k), ("p50_ms", "p99_ms")) for k in po if k != "rate_per_s"}}
        ti = sv.get("tight_tolerance")
        if ti:
            h["serving"]["tight"] = {"rtol": ti["rtol"], "requests": ti["requests"],
                                     "speedup": ti.get("speedup_solves_per_s"),
                                     **{k: form(ti.get(k), ("solves_per_s", "mean_iters"))
                                        for k in ("batched_f32", "one_at_a_time_f64")}}
    else:
        h["serving"] = None
    pr = out.get("precision")
    if pr:
        sig3 = lambda x: float(f"{x:.2e}") if isinstance(x, float) else x
        pair = lambda e: [sig3(e.get("rel")), sig3(e.get("max_block_rel"))] if e else None
        h["precision"] = {
            "f32_speedup_step": pr.get("f32_speedup_step"),
            "f32_vs_f64_legend": "[rel Frobenius, max block rel] vs the FP64 oracle: X, Dinv after 1, 2 SYNC sweeps; "
                                 "z: SYNC apply",
            "f32_vs_f64": {k: {"X1": pair(v.get("sweeps1", {}).get("X")), "D1": pair(v.get("sweeps1", {}).get("Dinv")),
                               "X2": pair(v.get("sweeps2", {}).get("X")), "D2": pair(v.get("sweeps2", {}).get("Dinv")),
                               "z": pair(v.get("apply"))}
                           for k, v in (pr.get("f32_vs_f64") or {}).items()}}
    else:
        h["precision"] = None
    ch = out.get("chunked")
    if ch:
        h["chunked_over_async_step_time"] = {k: v.get("chunk_over_async_step_time") for k, v in ch.items()}
    ws = out.get("warm_start")
    if ws:
        t = ws.get("totals") or {}
        h["warm_start_iters"] = {k: v.get("iters") for k, v in t.items()}
    fc = out.get("factor_convergence")
    if fc:
        h["factor_convergence"] = fc.get("summary")
    for k in ("max_rel_true_residual", "ilu_residual", "serving"):
        h[k] = _sig(h.get(k))
    h["factor_convergence"] = _sig(h.get("factor_convergence"), 3)
    oc = (h.get("cpu_baseline") or {}).get("oracle_check")
    if oc:
        if oc.get("f64_bitwise_equal"):
            oc = {k: v for k, v in oc.items() if k != "f64"}   # all zeros when bitwise equal
        h["cpu_baseline"]["oracle_check"] = _sig(oc)
    h["detail_file"] = detail_path
    h["source_hash"] = out.get("source_hash")
    return h


def summarize_main(argv):
    """bench.py --summarize-stats DIR TITLE COMMAND OUT.md
       bench.py --summarize-traffic FETCH_DIR WRITE_DIR COMMAND OUT_BASENAME  (writes .txt and .md)
       bench.py --summarize-serving-traffic FETCH_DIR WRITE_DIR FETCH_FACTOR WRITE_FACTOR COMMAND OUT.md
       bench.py --summarize-launch-traffic FETCH_DIR WRITE_DIR FETCH_FACTOR WRITE_FACTOR TITLE COMMAND OUT.md
       bench.py --summarize-trace-segments DIR MARKER_KERNEL TITLE COMMAND OUT.md SEGMENT_TITLE...
    Turn rocprofv3 output into the summaries kept under profiles/."""
    if argv[0] == "--summarize-stats":
        d, title, command, out = argv[1:5]
        open(out, "w").write(summarize_stats(d, title, command))
    elif argv[0] == "--summarize-trace-segments":
        d, marker, title, command, out = argv[1:6]
        open(out, "w").write(summarize_trace_segments(d, marker, title, command, argv[6:]))
    elif argv[0] == "--summarize-launch-traffic":
        fd, wd, cf, cw, title, command, out = argv[1:8]
        open(out, "w").write(summarize_launch_traffic(fd, wd, float(cf), float(cw), title, command))
    elif argv[0] == "--summarize-serving-traffic":
        fd, wd, cf, cw, command, out = argv[1:7]
        open(out, "w").write(summarize_serving_traffic(fd, wd, float(cf), float(cw), command))
    else:
        fd, wd, command, base = argv[1:5]
        js, md = summarize_traffic(fd, wd, command)
        open(base + ".txt", "w").write(js)
        open(base + ".md", "w").write(md)


if __name__ == "__main__":
    main()
