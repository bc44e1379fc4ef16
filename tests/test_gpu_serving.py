"""The serving form (include/abilu_serve.h): continuous batching of FGMRES solves.

* isolation: every request's solution and counters are the same alone, in a mix admitted at
  once, in a mix arriving while others are mid-solve, and under a pool so small that admission
  waits for memory. SYNC sweeps are deterministic, so "the same" is bitwise; the served result is
  also bitwise the one abilu_factor + fgmres_solve give for the same generated system.
  ASYNC sweeps update in place (rounding depends on scheduling): both runs converge, iteration
  counts agree within one, and the two solutions differ by less than the two residual bounds allow,
  ||A (x_mix - x_alone)|| <= 2 rtol ||b||.
* oracle: the served solution's true residual recomputed by the oracle SpMV on the downloaded
  system equals the reported one, and the oracle FGMRES on the oracle's synchronous factor of the
  same system takes the same number of iterations (within one).
* admission: the footprints of requests in the pool at the same time never exceed it; a request
  larger than the pool fails alone with ABILU_ENOMEM.
"""
import numpy as np
import pytest

import oracle
from paper_1912_00539_amd import workloads as W
from tests.dense_ref import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MIX = [
    dict(kind="tri", nx=24, ny=17, cfl=50.0, seed=101),
    dict(kind="aniso", nx=30, ny=12, cfl=300.0, seed=102),
    dict(kind="tri", nx=5, ny=3, cfl=10.0, seed=103),
    dict(kind="aniso", nx=1, ny=1, cfl=10.0, seed=104),
    dict(kind="tri", nx=1, ny=1, cfl=500.0, seed=105),
    dict(kind="tri", nx=60, ny=40, cfl=900.0, seed=106),
    dict(kind="aniso", nx=64, ny=32, cfl=20.0, seed=107),
    dict(kind="tri", nx=33, ny=33, cfl=200.0, seed=108),
    dict(kind="aniso", nx=7, ny=50, cfl=700.0, seed=109),
    dict(kind="tri", nx=90, ny=11, cfl=30.0, seed=110),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_00539_amd import abilu
    abilu.lib()
    yield
    torch.cuda.synchronize()


def L():
    from paper_1912_00539_amd import abilu
    return abilu


def dev():
    return torch.device("cuda:0")


def cfg_of(prec, mode, fsw, nsw=3, restart=10, maxit=60, rtol=1e-6, max_active=16):
    return L().serve_config(prec=prec, mode=mode, factor_sweeps=fsw, apply_sweeps=nsw, restart=restart, maxit=maxit,
                            rtol=rtol, max_active=max_active)


def pool_for(cfg, reqs, factor=None, minimum=0):
    need = [L().abilu_serve_footprint(cfg, r) for r in reqs]
    nbytes = int(max(need) * factor) if factor else sum(need) + (1 << 20)
    nbytes = max(nbytes, minimum)
    return torch.empty((nbytes + 255) // 256 * 256, dtype=torch.uint8, device=dev())


def serve(cfg, reqs, arrivals=None, pool=None):
    """(results, x tensors) of one server run over `reqs`."""
    xs = [torch.full((4 * L().abilu_gen_sizes(r)[0],), float("nan"), dtype=torch.float64, device=dev()) for r in reqs]
    srv = L().Server(cfg, pool if pool is not None else pool_for(cfg, reqs))
    try:
        res, _ = srv.run(reqs, arrivals=arrivals, x_outs=xs)
    finally:
        srv.destroy()
    torch.cuda.synchronize()
    return res, xs


def generated(req):
    """The request's system as generated on the device (tensors)."""
    n, z = L().abilu_gen_sizes(req)
    rowptr = torch.empty(n + 1, dtype=torch.int32, device=dev())
    colidx = torch.empty(z, dtype=torch.int32, device=dev())
    A = torch.empty(z * 16, dtype=torch.float64, device=dev())
    b = torch.empty(4 * n, dtype=torch.float64, device=dev())
    scratch = torch.empty(L().abilu_gen_scratch_bytes(req), dtype=torch.uint8, device=dev())
    L().abilu_gen_build(req, rowptr, colidx, A, b, scratch)
    return n, z, rowptr, colidx, A, b


def single_path(req, prec, mode, fsw, nsw=3, restart=10, maxit=60, rtol=1e-6):
    """abilu_factor + fgmres_solve (zero initial guess) on the device-generated system."""
    lib = L()
    n, z, rowptr, colidx, A, b = generated(req)
    p = lib.abilu_build_pattern(n, rowptr, colidx)
    dt = torch.float32 if prec == "f32" else torch.float64
    LU = torch.zeros(z * 16, dtype=dt, device=dev())
    Dinv = torch.zeros(n * 16, dtype=dt, device=dev())
    work = torch.zeros(lib.abilu_workspace_bytes(p, prec, restart), dtype=torch.uint8, device=dev())
    lib.abilu_factor(p, A, LU, Dinv, prec, fsw, mode, work)
    x = torch.zeros(4 * n, dtype=torch.float64, device=dev())
    st, res = lib.fgmres_solve(p, A, b, x, restart, maxit, rtol, LU, Dinv, prec, nsw, mode, work, zero_guess=True)
    torch.cuda.synchronize()
    p.destroy()
    return st, res, x


def host_system(req):
    """The request's system from the host twin of the device generator (the oracle's input)."""
    c = W.request_case(req)
    return c.n, c.rowptr, c.colidx, c.vals, c.b


KEYS = ("status", "iters", "restarts", "converged", "reorth", "flags", "rel_true_residual")


def same(ra, xa, rb, xb):
    for k in KEYS:
        assert ra[k] == rb[k], (k, ra[k], rb[k])
    assert torch.equal(xa, xb)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_isolation_sync_bitwise(prec):
    cfg_alone = cfg_of(prec, "sync", 2, max_active=1)
    cfg_mix = cfg_of(prec, "sync", 2, max_active=16)
    alone, xa = serve(cfg_alone, MIX)
    # all at once
    mix, xm = serve(cfg_mix, MIX)
    # arriving while others are mid-solve (members at different Arnoldi steps share ticks)
    stag, xs = serve(cfg_mix, MIX, arrivals=[0.0015 * q for q in range(len(MIX))])
    # a pool that holds about two requests: admission waits for memory
    tight, xt = serve(cfg_mix, MIX, pool=pool_for(cfg_mix, MIX, factor=2.2))
    for q in range(len(MIX)):
        assert alone[q]["status"] in (0, 1, 2), alone[q]
        same(alone[q], xa[q], mix[q], xm[q])
        same(alone[q], xa[q], stag[q], xs[q])
        same(alone[q], xa[q], tight[q], xt[q])
    print("iters:", [r["iters"] for r in alone], "restarts:", [r["restarts"] for r in alone])
    assert sum(r["restarts"] > 1 for r in alone) >= 1   # restarts exercised


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_results_do_not_depend_on_the_pool_contents(prec):
    """Every request reads only what admission and its own ticks wrote: with the pool's bytes set to
    0xFF (NaN in either precision) beforehand, SYNC results are the bits of a zeroed pool, and ASYNC
    solves still converge with finite x."""
    cfg = cfg_of(prec, "sync", 2, max_active=16)
    runs = []
    for fill in (0xFF, 0x00):
        pool = pool_for(cfg, MIX)
        pool.fill_(fill)
        runs.append(serve(cfg, MIX, pool=pool))
    (ra, xa), (rb, xb) = runs
    for q in range(len(MIX)):
        assert ra[q]["status"] in (0, 1, 2) and ra[q]["flags"] == 0, ra[q]
        same(ra[q], xa[q], rb[q], xb[q])
    cfg = cfg_of(prec, "async", 1, rtol=1e-2, restart=30, maxit=300, max_active=16)
    pool = pool_for(cfg, MIX)
    pool.fill_(0xFF)
    res, xs = serve(cfg, MIX, pool=pool)
    for q in range(len(MIX)):
        assert res[q]["converged"] and res[q]["flags"] == 0 and bool(torch.isfinite(xs[q]).all()), res[q]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_served_equals_single_system_path(prec):
    """In SYNC mode the served solve is bitwise abilu_factor + fgmres_solve on the same system."""
    res, xs = serve(cfg_of(prec, "sync", 2, max_active=16), MIX)
    for q, req in enumerate(MIX):
        st, one, x = single_path(req, prec, "sync", 2)
        assert res[q]["status"] == st
        for k in ("iters", "restarts", "converged", "reorth", "flags", "rel_true_residual"):
            assert res[q][k] == one[k], (req, k, res[q][k], one[k])
        assert torch.equal(xs[q], x), req


def test_isolation_async_within_bounds():
    rtol = 1e-2
    reqs = [r for r in MIX] + [dict(kind="aniso", nx=120, ny=60, cfl=100.0, seed=120),
                               dict(kind="tri", nx=100, ny=70, cfl=1000.0, seed=121)]
    alone, xa = serve(cfg_of("f32", "async", 1, rtol=rtol, restart=30, maxit=300, max_active=1), reqs)
    mix, xm = serve(cfg_of("f32", "async", 1, rtol=rtol, restart=30, maxit=300, max_active=16), reqs,
                    arrivals=[0.001 * q for q in range(len(reqs))])
    for q, req in enumerate(reqs):
        a, m = alone[q], mix[q]
        assert a["converged"] and m["converged"], (req, a, m)
        assert a["rel_true_residual"] <= rtol and m["rel_true_residual"] <= rtol
        assert abs(a["iters"] - m["iters"]) <= 1
        n, rp, ci, A, b = host_system(req)
        d = xm[q].cpu().numpy() - xa[q].cpu().numpy()
        assert np.linalg.norm(oracle.spmv(n, rp, ci, A, d)) <= 2 * rtol * np.linalg.norm(b) * (1 + 1e-12)


@pytest.mark.parametrize("q", [0, 1, 5, 7])
def test_served_solution_against_oracle(q):
    req = MIX[q]
    res, xs = serve(cfg_of("f64", "sync", 2, restart=30, maxit=300), [req])
    r = res[0]
    n, rp, ci, A, b = host_system(req)
    x = xs[0].cpu().numpy()
    true = np.linalg.norm(b - oracle.spmv(n, rp, ci, A, x)) / np.linalg.norm(b)
    assert abs(true - r["rel_true_residual"]) <= 1e-10 * max(1.0, true)
    X, D, _ = oracle.factor_sync(n, rp, ci, A, 2)
    ref = oracle.fgmres(n, rp, ci, A, b, X, D, restart=30, maxit=300, rtol=1e-6, apply_nsw=3)
    assert r["converged"] == ref["converged"]
    if ref["converged"]:
        assert abs(r["iters"] - ref["iters"]) <= 1
        assert r["rel_true_residual"] <= 1e-6
        if r["iters"] == ref["iters"]:
            assert rel(x, ref["x"]) <= 1e-9


def test_admission_by_footprint():
    cfg = cfg_of("f32", "async", 1, rtol=1e-2, restart=30, maxit=300, max_active=64)
    reqs = MIX + [dict(kind="tri", nx=80, ny=80, cfl=100.0, seed=130 + q) for q in range(6)]
    fp = [L().abilu_serve_footprint(cfg, r) for r in reqs]
    pool = pool_for(cfg, reqs, factor=2.5)
    cap = pool.numel()
    huge = dict(kind="tri", nx=400, ny=400, cfl=100.0, seed=140)
    assert L().abilu_serve_footprint(cfg, huge) > cap
    res, xs = serve(cfg, reqs + [huge], pool=pool)
    assert res[-1]["status"] == L().ABILU_ENOMEM
    for r, f in zip(res[:-1], fp):
        assert r["status"] == 0 and r["converged"] and r["footprint_bytes"] == f
        assert r["t_arrival"] <= r["t_admit"] <= r["t_done"]
    # at every admission instant, the requests holding memory fit in the pool
    ev = [(r["t_admit"], r["t_done"], r["footprint_bytes"]) for r in res[:-1]]
    for t, _, _ in ev:
        held = sum(f for a, d, f in ev if a <= t < d)
        assert held <= cap
    assert max(sum(1 for a, d, _ in ev if a <= t < d) for t, _, _ in ev) >= 2   # they did overlap


def test_submit_step_poll_api():
    lib = L()
    cfg = cfg_of("f64", "sync", 2, max_active=4)
    reqs = MIX[:6]
    srv = lib.Server(cfg, pool_for(cfg, reqs))
    xs = [torch.zeros(4 * lib.abilu_gen_sizes(r)[0], dtype=torch.float64, device=dev()) for r in reqs]
    ids = [srv.submit(r, x) for r, x in zip(reqs, xs)]
    assert srv.poll(ids[0]) is None
    ticks = 0
    while any(srv.poll(i) is None for i in ids):
        active, queued = srv.step()
        assert active <= 4
        ticks += 1
        assert ticks < 10000
    out = [srv.poll(i) for i in ids]
    srv.destroy()
    alone, xa = serve(cfg_of("f64", "sync", 2, max_active=1), reqs)
    for q in range(len(reqs)):
        same(alone[q], xa[q], out[q], xs[q])


def test_edge_cases():
    lib = L()
    # empty trace
    srv = lib.Server(cfg_of("f64", "sync", 1), pool_for(cfg_of("f64", "sync", 1), MIX[:1]))
    res, el = srv.run([])
    assert res == []
    srv.destroy()
    # maxit = 0: finished at the factor step with x = 0
    res, xs = serve(cfg_of("f32", "async", 1, maxit=0), MIX[:3])
    for r, x in zip(res, xs):
        assert r["iters"] == 0 and r["status"] == lib.ABILU_WARN_NOCONV and not r["converged"]
        assert torch.count_nonzero(x).item() == 0
        assert abs(r["rel_true_residual"] - 1.0) < 1e-15
    # no preconditioner and no factor sweeps
    res, xs = serve(cfg_of("f64", "sync", 0, nsw=0, restart=30, maxit=300, rtol=1e-3), MIX[:3])
    for q, r in enumerate(res):
        st, one, x = single_path(MIX[q], "f64", "sync", 0, nsw=0, restart=30, maxit=300, rtol=1e-3)
        assert r["iters"] == one["iters"] and torch.equal(xs[q], x)
    # one sweep of each kind
    for mode in ("sync", "async"):
        res, xs = serve(cfg_of("f64", mode, 1, nsw=1, restart=30, maxit=300, rtol=1e-3), MIX[:4])
        for q, r in enumerate(res):
            st, one, x = single_path(MIX[q], "f64", mode, 1, nsw=1, restart=30, maxit=300, rtol=1e-3)
            if mode == "sync":
                assert r["iters"] == one["iters"] and torch.equal(xs[q], x)
            else:
                assert r["converged"] == one["converged"]
    # invalid spec fails alone
    res, xs = serve(cfg_of("f64", "sync", 2), [MIX[0]], pool=pool_for(cfg_of("f64", "sync", 2), [MIX[0]]))
    srv = lib.Server(cfg_of("f64", "sync", 2), pool_for(cfg_of("f64", "sync", 2), [MIX[0]]))
    out, _ = srv.run([MIX[0], dict(kind="tri", nx=0, ny=3, cfl=1.0, seed=0)])
    srv.destroy()
    assert out[1]["status"] == lib.ABILU_EINVAL and out[0]["iters"] == res[0]["iters"]


def test_stats_bytes_match_single_system_profile():
    """The server's algorithmic byte count equals the single-system path's per-launch byte model
    (the library profile of abilu_factor + fgmres_solve) over the same requests (SYNC: the same
    iterations and Gram-Schmidt decisions), plus the one normalisation of V_0 the server does
    ahead at the last cycle end of each request (read and write of 4N doubles)."""
    lib = L()
    reqs = MIX[:5]
    cfg = cfg_of("f64", "sync", 2, restart=10, maxit=60)
    srv = lib.Server(cfg, pool_for(cfg, reqs))
    res, _ = srv.run(reqs)
    st = srv.stats()
    srv.destroy()
    assert st["admitted"] == len(reqs) and st["retired"] == len(reqs) and st["ticks"] > 0
    lib.abilu_profile_enable(True, 100000)
    for req in reqs:
        single_path(req, "f64", "sync", 2)
    rep = lib.abilu_profile_report()
    lib.abilu_profile_enable(False)
    single = sum(v[2] for k, v in rep.items() if not k.startswith(("_", "gen_")))   # generation not counted
    ahead = sum(64.0 * r["n"] for r in res if r["iters"] > 0)
    assert abs(st["bytes"] - (single + ahead)) <= 1e-9 * single, (st["bytes"], single, ahead)
