"""Chunked sweeps on the GPU (Gauss-Seidel within chunks of consecutive rows, the schedule of the
paper's OpenMP chunks, Section 3.3) against the CPU FP64 oracle, through the C ABI.

  * chunk schedules (integers): bit-exact against the oracle's dependence levels of each chunk's
    diagonal block of the pattern;
  * ABILU_CHUNK_SYNC (deterministic) against oracle.factor_chunked / oracle.apply_chunked:
    double precision 1e-12, or 8x the oracle's own sensitivity to a one-ulp perturbation of A
    where that is larger; single precision 1e-5, or 8x the sensitivity to rounding A to float;
  * ABILU_CHUNK_ASYNC (in place, nondeterministic across chunks): pinned where its result is
    unique -- one chunk over all rows gives the sequential ILU(0) and the exact substitutions in
    one sweep, and any chunking is exact after as many sweeps as there are chunks.
"""
import numpy as np
import pytest

import oracle
from paper_1912_00539_amd import workloads as W
from tests.dense_ref import assert_same_bits, rel
from tests.f32_bars import FactorBars, VectorBars, perturb, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_00539_amd import abilu
    abilu.lib()
    yield
    torch.cuda.synchronize()


def DS(case, prec="f64", restart=30, R=None, runner="auto"):
    from paper_1912_00539_amd.runtime import DeviceSystem
    s = DeviceSystem(case, prec=prec, restart=restart)
    if R is not None:
        s.set_chunks(R, runner)
    return s


RUNNERS = ["levels", "rows"]


CASES = {
    "quad32": lambda: W.case("quad32"),
    "tri40x30_rcm": lambda: W.case("tri", seed=3, nx=40, ny=30, order="rcm", shift="cfl", cfl=100.0),
    "nine23x17": lambda: W.case("nine", seed=4, nx=23, ny=17),
    "random1000": lambda: W.case("random", seed=5, n=1000, deg=5.0, order="random"),
    "aniso50x20_line": lambda: W.case("aniso", seed=6, nx=50, ny=20, order="line", shift="cfl", cfl=100.0),
    "chain7": lambda: W.case("chain", seed=7, n=7),
    "single": lambda: W.case("chain", seed=8, n=1),
}
NAMES = list(CASES)
RS = [1, 3, 64, 256, 4096]


def get(name):
    return CASES[name]()


def chunk_levels(c, R):
    """Per-row levels inside each chunk: the oracle's triangular levels of the pattern with every
    block outside the chunks' diagonal blocks removed."""
    rows = np.repeat(np.arange(c.n), np.diff(c.rowptr))
    keep = (rows // R) == (c.colidx // R)
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=c.n))]).astype(np.int32)
    ci = c.colidx[keep].astype(np.int32)
    _, _, lo, up = oracle.levels(c.n, rp, ci)
    return lo, up


# ------------------------------------------------------------------ schedule (integers, bit-exact)
@pytest.mark.parametrize("R", RS)
@pytest.mark.parametrize("name", NAMES)
def test_chunk_schedule_bit_exact(name, R):
    from paper_1912_00539_amd import abilu as L
    c = get(name)
    s = DS(c)
    info = s.set_chunks(R)
    nch = (c.n + R - 1) // R
    lo, up = chunk_levels(c, R)
    assert info["rows_per_chunk"] == R and info["nchunks"] == nch
    for upper, lev in ((0, lo), (1, up)):
        tot = info["levels_upper" if upper else "levels_lower"]
        order = torch.zeros(max(c.n, 1), dtype=torch.int32, device="cuda")
        lvptr = torch.zeros(nch + 1, dtype=torch.int32, device="cuda")
        lvstart = torch.zeros(tot + nch, dtype=torch.int32, device="cuda")
        L.abilu_pattern_chunk_export(s.pattern, upper, order, lvptr, lvstart)
        torch.cuda.synchronize()
        order, lvptr, lvstart = order.cpu().numpy()[: c.n], lvptr.cpu().numpy(), lvstart.cpu().numpy()
        nl_chunk = [int(lev[q * R:min(c.n, (q + 1) * R)].max()) for q in range(nch)]
        np.testing.assert_array_equal(np.diff(lvptr), np.array(nl_chunk) + 1)
        assert lvptr[0] == 0 and lvptr[-1] == tot + nch
        assert info["max_levels_upper" if upper else "max_levels_lower"] == max(nl_chunk)
        for q in range(nch):
            c0, c1 = q * R, min(c.n, (q + 1) * R)
            st = lvstart[lvptr[q]:lvptr[q + 1]]
            assert st[0] == c0 and st[-1] == c1
            for lv in range(nl_chunk[q]):
                got = order[st[lv]:st[lv + 1]]
                want = c0 + np.nonzero(lev[c0:c1] == lv + 1)[0]
                np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["tri40x30_rcm", "aniso50x20_line", "random1000", "nine23x17"])
def test_runners_agree_bitwise(name, prec):
    """CHUNK_SYNC gives the same bits whether a chunk runs level by level in a workgroup or row by
    row in one quad: each row reads the same values either way."""
    c = get(name)
    r = np.random.default_rng(8).uniform(-1, 1, 4 * c.n)
    out = {}
    for runner in RUNNERS:
        s = DS(c, prec, R=64, runner=runner)
        assert s.set_chunks(64, runner)["runner"] == runner
        s.factor(2, "chunk_sync")
        X, D = s.factor_host()
        rt = torch.from_numpy(r).cuda()
        zt = torch.zeros_like(rt)
        s.apply(rt, zt, 3, "chunk_sync")
        out[runner] = (X, D, zt.cpu().numpy())
    for a, b in zip(out["levels"], out["rows"]):
        np.testing.assert_array_equal(a, b)


def test_auto_runner_choice():
    """AUTO takes one quad per chunk for chains (line-ordered wall layers: one row per level) and a
    workgroup per chunk where a chunk's rows are mostly independent (RCM-ordered triangles)."""
    assert DS(get("aniso50x20_line"), R=64).set_chunks(64)["runner"] == "rows"
    assert DS(get("tri40x30_rcm"), R=64).set_chunks(64)["runner"] == "levels"


def test_chunk_schedule_replaced_and_modes_need_it():
    from paper_1912_00539_amd import abilu as L
    c = get("nine23x17")
    s = DS(c)
    with pytest.raises(L.AbiluError) as ei:
        s.factor(1, "chunk_sync")
    assert ei.value.status == L.ABILU_EINVAL
    for bad in (0, -3, 4097):
        with pytest.raises(L.AbiluError):
            L.abilu_pattern_set_chunks(s.pattern, bad)
    assert L.lib().abilu_pattern_set_chunks(s.pattern.handle, 64, 3, L._stream(None)) == L.ABILU_EINVAL
    assert s.set_chunks(50)["nchunks"] == 8
    assert s.set_chunks(400)["nchunks"] == 1


# ------------------------------------------------------------------ CHUNK_SYNC factor vs the oracle
def check_chunked(c, nsw, R, prec, X, D, what=""):
    """FP64: bit for bit against the chunked oracle (the GPU's block products and inverse evaluate
    the oracle's operations in its order, and the Gauss-Seidel order within a chunk is the oracle's
    row-major order). FP32: block by block (tests/f32_bars.py)."""
    run = lambda A, X0, k=nsw: oracle.factor_chunked(c.n, c.rowptr, c.colidx, A, k, R, X0=X0)[:2]
    if prec == "f64":
        Xo, Do = run(c.vals, None)
        assert_same_bits(X, Xo, f"{what} X")
        assert_same_bits(D, Do, f"{what} Dinv")
        return None

    def perturbed(g):
        # A and every iterate stored between sweeps perturbed by a float ulp
        Ap = perturb(c.vals, g)
        Xp = None
        for _ in range(nsw):
            Xp, _ = run(Ap, Xp, 1)
            Xp = perturb(Xp, g)
        return run(Ap, Xp, 0)
    out = FactorBars(run, c.vals, perturbed=perturbed).check(X, D, what)
    report(f"{what} f32 chunked", out)
    return out


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("nsw", [1, 2, 3])
@pytest.mark.parametrize("R", RS)
@pytest.mark.parametrize("name", NAMES)
def test_factor_chunk_sync_f64(name, R, nsw, runner):
    c = get(name)
    s = DS(c, "f64", R=R, runner=runner)
    s.factor(nsw, "chunk_sync")
    X, D = s.factor_host()
    check_chunked(c, nsw, R, "f64", X, D, name)
    assert s.flags() == 0


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("nsw", [1, 3])
@pytest.mark.parametrize("R", [3, 64])
@pytest.mark.parametrize("name", NAMES)
def test_factor_chunk_sync_f32(name, R, nsw, runner):
    c = get(name)
    s = DS(c, "f32", R=R, runner=runner)
    s.factor(nsw, "chunk_sync")
    X, D = s.factor_host()
    check_chunked(c, nsw, R, "f32", X, D, name)


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("name", ["nine23x17", "tri40x30_rcm", "random1000"])
def test_factor_chunk_sync_warm_start(name, runner):
    """INIT_FROM_LU continues the chunked iteration: p sweeps then q sweeps equal p + q sweeps."""
    c = get(name)
    for prec in ("f64", "f32"):
        for first, second in ((1, 2), (2, 1)):
            s = DS(c, prec, R=64, runner=runner)
            s.factor(first, "chunk_sync")
            s.factor(second, "chunk_sync", init="LU")
            X, D = s.factor_host()
            check_chunked(c, first + second, 64, prec, X, D, f"{name} {first}+{second}")


# ------------------------------------------------------------------ CHUNK_ASYNC factor: unique results
def check_sequential(c, prec, X, D, what=""):
    """Against the sequential block ILU(0): FP64 bit for bit (every block is then computed from
    final values by the oracle's operations), FP32 block by block."""
    run = lambda A, X0: oracle.ilu0_seq(c.n, c.rowptr, c.colidx, A)[:2]
    if prec == "f64":
        Xs, Ds = run(c.vals, None)
        assert_same_bits(X, Xs, f"{what} X")
        assert_same_bits(D, Ds, f"{what} Dinv")
    else:
        report(f"{what} f32 vs sequential ILU(0)", FactorBars(run, c.vals).check(X, D, what))


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", NAMES)
def test_factor_single_chunk_is_sequential_ilu(name, prec, runner):
    """One chunk over every row: one sweep is the sequential block ILU(0) in both chunked modes,
    and the two modes (the same kernel reading only the chunk's own rows) agree bit for bit."""
    c = get(name)
    out = []
    for mode in ("chunk_sync", "chunk_async"):
        s = DS(c, prec, R=4096, runner=runner)
        s.factor(1, mode)
        X, D = s.factor_host()
        check_sequential(c, prec, X, D, f"{name} {mode}")
        out.append((X, D))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("name,R", [("nine23x17", 64), ("random1000", 128), ("chain7", 2),
                                    ("aniso50x20_line", 256), ("tri40x30_rcm", 512)])
def test_factor_chunked_exact_after_one_sweep_per_chunk(name, R, runner):
    """Section 4.2: exact after as many sweeps as chunks, whatever the order in which the chunks
    ran (CHUNK_ASYNC) -- and CHUNK_SYNC likewise."""
    c = get(name)
    nch = (c.n + R - 1) // R
    for mode in ("chunk_async", "chunk_sync"):
        s = DS(c, "f64", R=R, runner=runner)
        s.factor(nch, mode)
        X, D = s.factor_host()
        check_sequential(c, "f64", X, D, f"{name} {mode}")
        assert s.ilu_residual() <= 1e-12


@pytest.mark.parametrize("name", ["tri40x30_rcm", "nine23x17", "aniso50x20_line"])
def test_factor_chunk_async_residual(name):
    """CHUNK_ASYNC is nondeterministic across chunks: its ILU residual is finite, decreases with
    the sweep count, and is reported beside CHUNK_SYNC's (the oracle's) and the unchunked
    asynchronous sweeps' at the same sweep count."""
    c = get(name)
    out = []
    for nsw in (1, 2, 3):
        a = DS(c, "f64", R=64)
        a.factor(nsw, "chunk_async")
        ra = a.ilu_residual()
        Xo, _, _ = oracle.factor_chunked(c.n, c.rowptr, c.colidx, c.vals, nsw, 64)
        rs = oracle.ilu_residual(c.n, c.rowptr, c.colidx, c.vals, Xo)
        b = DS(c, "f64")
        b.factor(nsw, "async")
        assert np.isfinite(ra)
        out.append((nsw, ra, rs, b.ilu_residual()))
    print("nsw, chunk_async, chunk_sync (oracle), async:", out)
    assert out[-1][1] < out[0][1]


# ------------------------------------------------------------------ apply
@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("nsw", [1, 2, 3])
@pytest.mark.parametrize("R", RS)
@pytest.mark.parametrize("name", NAMES)
def test_apply_chunk_sync_f64(name, R, nsw, runner):
    c = get(name)
    s = DS(c, "f64", R=R, runner=runner)
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 2)
    s.set_factor(Xo, Do)
    r = np.random.default_rng(nsw).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, nsw, "chunk_sync")
    ref = oracle.apply_chunked(c.n, c.rowptr, c.colidx, Xo, Do, r, nsw, R)
    assert_same_bits(zt.cpu().numpy(), ref, "z")


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("nsw", [1, 3])
@pytest.mark.parametrize("name", NAMES)
def test_apply_chunk_sync_f32(name, nsw, runner):
    c = get(name)
    s = DS(c, "f32", R=64, runner=runner)
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 1)
    X = Xo.astype(np.float32).astype(np.float64)   # the oracle factor as FP32 storage holds it
    D = Do.astype(np.float32).astype(np.float64)
    s.set_factor(X, D)
    r = np.random.default_rng(10 + nsw).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, nsw, "chunk_sync")
    bars = VectorBars(lambda X_, D_, r_: oracle.apply_chunked(c.n, c.rowptr, c.colidx, X_, D_, r_, nsw, 64), X, D, r)
    e, worst = bars.check(zt.cpu().numpy(), name)
    print(f"{name} f32 chunked apply {nsw}: rel {e:.2e}, worst cell at {worst:.2f} of its bar")


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("name,R", [("quad32", 4096), ("tri40x30_rcm", 4096), ("aniso50x20_line", 4096),
                                    ("random1000", 4096), ("chain7", 2), ("aniso50x20_line", 256),
                                    ("nine23x17", 64)])
def test_apply_chunked_exact(name, R, runner):
    """One chunk: one sweep pair is the exact forward and backward substitution (Algorithm 1);
    any chunking: exact after as many sweeps as chunks; both modes."""
    c = get(name)
    nch = (c.n + R - 1) // R
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    r = np.random.default_rng(2).uniform(-1, 1, 4 * c.n)
    ref = oracle.trisolve_exact(c.n, c.rowptr, c.colidx, Xs, Ds, r)
    s = DS(c, "f64", R=R, runner=runner)
    s.set_factor(Xs, Ds)
    rt = torch.from_numpy(r).cuda()
    for mode in ("chunk_sync", "chunk_async"):
        zt = torch.zeros_like(rt)
        s.apply(rt, zt, nch, mode)
        assert_same_bits(zt.cpu().numpy(), ref, mode)


def test_apply_chunk_async_converges():
    c = get("aniso50x20_line")
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    r = np.random.default_rng(3).uniform(-1, 1, 4 * c.n)
    ref = oracle.trisolve_exact(c.n, c.rowptr, c.colidx, Xs, Ds, r)
    s = DS(c, "f64", R=64)
    s.set_factor(Xs, Ds)
    rt = torch.from_numpy(r).cuda()
    errs = []
    for nsw in (1, 2, 4):
        zt = torch.zeros_like(rt)
        s.apply(rt, zt, nsw, "chunk_async")
        e = rel(zt.cpu().numpy(), ref)
        e_sync = rel(oracle.apply_chunked(c.n, c.rowptr, c.colidx, Xs, Ds, r, nsw, 64), ref)
        e_jac = rel(oracle.apply_sync(c.n, c.rowptr, c.colidx, Xs, Ds, r, nsw), ref)
        assert np.isfinite(e)
        errs.append((nsw, e, e_sync, e_jac))
    print("nsw, chunk_async error, chunk_sync error (oracle), Jacobi error (oracle):", errs)
    assert errs[-1][1] < errs[0][1]


# ------------------------------------------------------------------ FGMRES with the chunked preconditioner
@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("mode", ["chunk_sync", "chunk_async"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["quad32", "tri40x30_rcm", "aniso50x20_line"])
def test_fgmres_chunked(name, prec, mode, runner):
    c = get(name)
    s = DS(c, prec, restart=30, R=64, runner=runner)
    s.factor(1, mode)
    st, res = s.solve(apply_sweeps=3, mode=mode, rtol=1e-6, maxit=300)
    x = s.x.cpu().numpy()
    rt = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    assert st == 0 and res["converged"], res
    assert rt <= 1e-6 and abs(rt - res["rel_true_residual"]) <= 1e-10 * max(1.0, rt) + 1e-14


# ------------------------------------------------------------------ full size
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_size_tri300_chunk_sync(prec):
    """180,000 triangles (CFL 100, random permutation + RCM), 64-row chunks: factor (1 and 2
    sweeps) and apply (2 sweeps) against the oracle over every block and entry."""
    c = W.case("tri300")
    for nsw in (1, 2):
        s = DS(c, prec, R=64)
        s.factor(nsw, "chunk_sync")
        X, D = s.factor_host()
        check_chunked(c, nsw, 64, prec, X, D, f"tri300 {nsw}")
    Xo, Do, _ = oracle.factor_chunked(c.n, c.rowptr, c.colidx, c.vals, 2, 64)
    if prec == "f32":   # the oracle factor as FP32 storage holds it
        Xo, Do = Xo.astype(np.float32).astype(np.float64), Do.astype(np.float32).astype(np.float64)
    s.set_factor(Xo, Do)
    r = np.random.default_rng(5).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, 2, "chunk_sync")
    run = lambda X_, D_, r_: oracle.apply_chunked(c.n, c.rowptr, c.colidx, X_, D_, r_, 2, 64)
    if prec == "f64":
        assert_same_bits(zt.cpu().numpy(), run(Xo, Do, r), "z")
    else:
        VectorBars(run, Xo, Do, r).check(zt.cpu().numpy(), "tri300")


def test_full_size_aniso1000_line_chunk_sync():
    """500,000 anisotropic quads in line order (each 64-row chunk is one dependency chain along
    the wall-normal line): one FP64 chunked sweep against the oracle, with its rounding
    sensitivity bound, and the FP32 chunked preconditioner inside FGMRES."""
    c = W.case("aniso1000", order="line")
    s = DS(c, "f64", R=64)
    s.factor(1, "chunk_sync")
    X, D = s.factor_host()
    check_chunked(c, 1, 64, "f64", X, D, "aniso1000 line")
    s32 = DS(c, "f32", restart=30, R=64)
    s32.factor(1, "chunk_async")
    st, res = s32.solve(apply_sweeps=3, mode="chunk_async", rtol=1e-2, maxit=300)
    assert st == 0 and res["converged"]


def test_full_size_aniso1000_line_runners_agree_f32():
    """The bench's chunked case (500,000 quads in line order, 16-row chunks, FP32): the quad-per-chunk
    runner (its pipelined form: every row has at most two lower and two upper blocks and two
    update pairs) gives the bits of the workgroup-per-chunk runner for three CHUNK_SYNC factor
    sweeps (the first from A) and for three apply sweep pairs."""
    c = W.case("aniso1000", order="line")
    r = np.random.default_rng(9).uniform(-1, 1, 4 * c.n)
    out = {}
    for runner in RUNNERS:
        s = DS(c, "f32", R=16, runner=runner)
        assert s.set_chunks(16, runner)["runner"] == runner
        s.factor(3, "chunk_sync")
        X, D = s.factor_host()
        rt = torch.from_numpy(r).cuda()
        zt = torch.zeros_like(rt)
        s.apply(rt, zt, 3, "chunk_sync")
        out[runner] = (X, D, zt.cpu().numpy())
        del s
    for a, b, what in zip(out["levels"], out["rows"], ("X", "Dinv", "z")):
        np.testing.assert_array_equal(a, b, err_msg=what)


# ------------------------------------------------------------------ orderings + chunked sweeps, end to end
def test_line_ordering_then_chunked_sweeps():
    """Section 5 with the chunk schedule of Section 3.3: the library finds lines on a boundary-layer
    mesh from its geometric couplings and orders it line-RCM (and RCM for comparison), both equal
    to the ordering oracle's bit for bit; the same seeded matrix is assembled in each of the
    oracle's orders. One CHUNK_SYNC FP64 sweep (16-row chunks) matches
    the chunked oracle; under line-RCM each chunk runs along a wall-normal line and its ILU residual
    is well below RCM's (2.3e-3 against 9.6e-3 in the oracle for this case). An asynchronous
    chunked FP32 solve then converges, its true residual confirmed by the oracle SpMV."""
    from paper_1912_00539_amd import abilu as L
    m = W.aniso_quad_mesh(60, 40)
    base = W.natural_order(m)
    c0 = W.assemble(m, base, 3, "cfl", cfl=100.0)
    w = W.block_face_weights(m, base, c0.rowptr, c0.colidx)
    from oracle import orderings as O
    lo, lp, nl = L.abilu_find_lines(c0.n, c0.rowptr, c0.colidx, w, 10.0, 4.0)
    olo, olp, onl = O.find_lines(c0.n, c0.rowptr, c0.colidx, w, 10.0, 4.0)
    assert nl == onl == 60
    np.testing.assert_array_equal(lo, olo)
    np.testing.assert_array_equal(lp, olp)
    res = {}
    for name in ("rcm", "line_rcm"):
        new = L.abilu_order(c0.n, c0.rowptr, c0.colidx, name, lo, lp).astype(np.int64)
        onew = O.rcm(c0.n, c0.rowptr, c0.colidx) if name == "rcm" else \
            O.hybrid_line_order(c0.n, c0.rowptr, c0.colidx, olo, olp, "rcm")
        np.testing.assert_array_equal(new, onew)
        c = W.assemble(m, onew, 3, "cfl", cfl=100.0)   # the oracle's ordering feeds both sides
        s = DS(c, "f64", R=16)
        s.factor(1, "chunk_sync")
        X, D = s.factor_host()
        check_chunked(c, 1, 16, "f64", X, D, name)
        Xo, _, _ = oracle.factor_chunked(c.n, c.rowptr, c.colidx, c.vals, 1, 16)
        res[name] = s.ilu_residual()
        assert abs(res[name] - oracle.ilu_residual(c.n, c.rowptr, c.colidx, c.vals, Xo)) <= 1e-10 * res[name]
        s32 = DS(c, "f32", restart=30, R=16)
        s32.factor(1, "chunk_async")
        st, r = s32.solve(apply_sweeps=3, mode="chunk_async", rtol=1e-6, maxit=300)
        x = s32.x.cpu().numpy()
        true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
        assert st == 0 and r["converged"] and true <= 1e-6, (name, r)
    print("ILU residual after one chunked sweep:", res)
    assert res["line_rcm"] < 0.5 * res["rcm"]
