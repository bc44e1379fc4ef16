"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars:
  * pattern analysis (integers): bit-exact;
  * double-precision synchronous factor sweeps and synchronous apply sweeps: bit-exact. The
    stated bar is 1e-12 relative; the GPU's double-precision block products evaluate every
    product and sum in the oracle's order without fused multiply-add, and its 4x4 inverse follows
    the oracle's elimination operation for operation, so the results are identical;
  * SpMV: 1e-13 (rounding order only: each block's four products are summed as one fused tree
    before the accumulator, which keeps the accumulator's dependent chain short);
  * single precision against the double oracle, block by block (tests/f32_bars.py): every block
    of X and Dinv (every cell of z) within max(1e-5, 32 s_b), s_b being that block's relative change
    in the oracle's result under a one-float-ulp perturbation of the inputs; checked against the
    oracle on A and on A rounded to float (arithmetic error apart from input rounding);
  * FGMRES: iteration counts within 1, true residual below rtol on both sides.
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


def DS(case, prec="f64", restart=30):
    from paper_1912_00539_amd.runtime import DeviceSystem
    return DeviceSystem(case, prec=prec, restart=restart)


def parity_cases():
    return {
        "quad32": lambda: W.case("quad32"),
        "tri40x30_rcm": lambda: W.case("tri", seed=3, nx=40, ny=30, order="rcm", shift="cfl", cfl=100.0),
        "nine23x17": lambda: W.case("nine", seed=4, nx=23, ny=17),
        "random1000": lambda: W.case("random", seed=5, n=1000, deg=5.0, order="random"),
        "aniso50x20_line": lambda: W.case("aniso", seed=6, nx=50, ny=20, order="line", shift="cfl", cfl=100.0),
        "chain7": lambda: W.case("chain", seed=7, n=7),
        "single": lambda: W.case("chain", seed=8, n=1),
    }


CASES = list(parity_cases().keys())


def get(name):
    return parity_cases()[name]()


# ------------------------------------------------------------------ pattern analysis (a1)
@pytest.mark.parametrize("name", CASES)
def test_pattern_bit_exact(name):
    _check_pattern(get(name))


def _check_pattern(c):
    """diag_pos, the update-set offsets and pair lists exported by the library equal the oracle's."""
    from paper_1912_00539_amd import abilu as L
    s = DS(c)
    n, z, npairs = s.pattern.info()
    ptr, pik, pkj = oracle.pairs(c.n, c.rowptr, c.colidx)
    assert (n, z, npairs) == (c.n, c.nnzb, int(ptr[-1]))
    dp = torch.zeros(max(c.n, 1), dtype=torch.int32, device="cuda")
    pp = torch.zeros(z + 1, dtype=torch.int32, device="cuda")
    a = torch.zeros(max(npairs, 1), dtype=torch.int32, device="cuda")
    b = torch.zeros(max(npairs, 1), dtype=torch.int32, device="cuda")
    L.abilu_pattern_export(s.pattern, dp, pp, a, b)
    torch.cuda.synchronize()
    diag = np.array([c.rowptr[i] + np.nonzero(c.colidx[c.rowptr[i]:c.rowptr[i + 1]] == i)[0][0] for i in range(c.n)])
    np.testing.assert_array_equal(dp.cpu().numpy()[: c.n], diag)
    np.testing.assert_array_equal(pp.cpu().numpy(), ptr)
    np.testing.assert_array_equal(a.cpu().numpy()[:npairs], pik)
    np.testing.assert_array_equal(b.cpu().numpy()[:npairs], pkj)


# chain lengths whose prefix scans end at, just before and just after a 2,048-entry scan tile:
# over the N rows (lower/upper offsets) and over the Z = 3N - 2 blocks (update-set offsets)
@pytest.mark.parametrize("n", [2047, 2048, 2049, 1365, 1366, 1367, 6145])
def test_pattern_and_factor_at_scan_tile_boundaries(n):
    c = W.case("chain", seed=n, n=n)
    _check_pattern(c)
    s = DS(c, "f64")
    s.factor(1, "sync")
    X, D = s.factor_host()
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 1)
    assert_same_bits(X, Xo, "X")
    assert_same_bits(D, Do, "Dinv")


def test_pattern_invalid_rejected():
    from paper_1912_00539_amd import abilu as L
    c = W.case("quad", nx=5, ny=4)
    for mutate in ("unsorted", "range", "nodiag", "rowptr"):
        rp = c.rowptr.copy(); ci = c.colidx.copy()
        if mutate == "unsorted":
            ci[[0, 1]] = ci[[1, 0]]
        elif mutate == "range":
            ci[5] = c.n + 3
        elif mutate == "nodiag":
            d = int(np.nonzero(ci[rp[2]:rp[3]] == 2)[0][0]) + rp[2]
            ci = np.delete(ci, d)                 # row 2 loses its diagonal block
            rp = rp.copy(); rp[3:] -= 1
        elif mutate == "rowptr":
            rp[3], rp[4] = rp[4], rp[3]
        with pytest.raises(L.AbiluError) as ei:
            L.abilu_build_pattern(c.n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda())
        assert ei.value.status == L.ABILU_EPATTERN, mutate


def test_empty_matrix():
    from paper_1912_00539_amd import abilu as L
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = L.abilu_build_pattern(0, rp, ci)
    assert p.info() == (0, 0, 0)
    work = torch.zeros(L.abilu_workspace_bytes(p, "f64", 5), dtype=torch.uint8, device="cuda")
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert L.abilu_factor(p, e, e, e, "f64", 3, "sync", work) == 0
    assert L.abilu_apply(p, e, e, "f64", e, e.clone(), 3, "sync", work) == 0
    st, res = L.fgmres_solve(p, e, e, e.clone(), 5, 10, 1e-2, e, e, "f64", 3, "sync", work, zero_guess=True)
    assert st == 0 and res["converged"] == 1


# ------------------------------------------------------------------ factor sweeps (a2-a4)
@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("nsw", [0, 1, 2, 3])
def test_factor_sync_f64(name, nsw):
    c = get(name)
    s = DS(c, "f64")
    s.factor(nsw, "sync")
    X, D = s.factor_host()
    Xo, Do, fo = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, nsw)
    assert_same_bits(X, Xo, "X")
    assert_same_bits(D, Do, "Dinv")
    assert s.flags() == fo == 0


def F32Bars(c, nsw, X0=None):
    """Block-by-block single-precision bars for nsw synchronous sweeps (tests/f32_bars.py): the
    sensitivity run perturbs A and every iterate between sweeps, sweep by sweep, the last one
    before its diagonal blocks are inverted."""
    sync = lambda A, X0_, k: oracle.factor_sync(c.n, c.rowptr, c.colidx, A, k, X0=X0_)[:2]

    def perturbed(g):
        Ap = perturb(c.vals, g)
        X = Ap if X0 is None else perturb(X0, g)
        for _ in range(nsw):
            X, _ = sync(Ap, X, 1)
            X = perturb(X, g)
        return sync(Ap, X, 0)
    return FactorBars(lambda A, X0_: sync(A, X0_, nsw), c.vals, X0, perturbed=perturbed)


def apply_bars(c, X, D, r, nsw):
    return VectorBars(lambda X_, D_, r_: oracle.apply_sync(c.n, c.rowptr, c.colidx, X_, D_, r_, nsw), X, D, r)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("nsw", [1, 3])
def test_factor_sync_f32(name, nsw):
    c = get(name)
    s = DS(c, "f32")
    s.factor(nsw, "sync")
    X, D = s.factor_host()
    report(f"{name} f32 {nsw} sweeps", F32Bars(c, nsw).check(X, D, name))


@pytest.mark.parametrize("name", ["quad32", "nine23x17", "random1000", "chain7"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_factor_exact_at_depth(name, prec):
    """Sync sweeps reach the sequential block ILU(0) at the dependency depth D (Lemma 2,
    Theorem 8); in-place asynchronous sweeps (one launch per sweep, so every read sees at least
    the previous sweep) reach the same floating-point fixed point bit for bit."""
    c = get(name)
    D, _ = oracle.depth(c.n, c.rowptr, c.colidx)
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    s = DS(c, prec)
    s.factor(D, "sync")
    Xg, Dg = s.factor_host()
    if prec == "f64":
        # at the depth every block is computed from final values by the oracle's operations
        assert_same_bits(Xg, Xs, "X")
        assert_same_bits(Dg, Ds, "Dinv")
    else:
        assert rel(Xg, Xs) <= 1e-5 and rel(Dg, Ds) <= 1e-5
    a = DS(c, prec)
    a.factor(D + 2, "async")
    Xa, Da = a.factor_host()
    np.testing.assert_array_equal(Xa, Xg)
    np.testing.assert_array_equal(Da, Dg)
    assert s.ilu_residual() <= (1e-13 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("name", ["tri40x30_rcm", "nine23x17"])
def test_factor_async_residual_reported(name):
    """ASYNC is nondeterministic: its ILU residual is reported (beside the Jacobi-type
    iteration's at the same sweep count), is finite and decreases with the sweep count."""
    c = get(name)
    out = []
    r0 = oracle.ilu_residual(c.n, c.rowptr, c.colidx, c.vals, c.vals)
    for nsw in (1, 2, 3):
        a = DS(c, "f64")
        a.factor(nsw, "async")
        ra = a.ilu_residual()
        Xo, _, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, nsw)
        rs = oracle.ilu_residual(c.n, c.rowptr, c.colidx, c.vals, Xo)
        assert np.isfinite(ra)
        out.append((nsw, ra, rs))
    print("nsw, async residual, sync residual:", out)
    assert out[0][1] < r0 and out[-1][1] < out[0][1]


@pytest.mark.parametrize("name", ["tri40x30_rcm", "nine23x17"])
def test_ilu_residual_matches_oracle(name):
    c = get(name)
    s = DS(c, "f64")
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 1)
    s.set_factor(Xo, Do)
    ref = oracle.ilu_residual(c.n, c.rowptr, c.colidx, c.vals, Xo)
    assert abs(s.ilu_residual() - ref) <= 1e-12 * ref


def test_factor_warm_start():
    """INIT_FROM_LU: sweeps continue from the factor in d_LU (x^{p+q} from x^p)."""
    c = get("nine23x17")
    for prec in ("f64", "f32"):
        for first, second in ((1, 2), (2, 1), (1, 0)):
            s = DS(c, prec)
            s.factor(first, "sync")
            s.factor(second, "sync", init="LU")
            X, D = s.factor_host()
            if prec == "f64":
                Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, first + second)
                assert_same_bits(X, Xo, f"X {first}+{second}")
                assert_same_bits(D, Do, f"Dinv {first}+{second}")
            else:
                F32Bars(c, first + second).check(X, D, f"{first}+{second}")


def test_factor_singular_and_nonfinite_flags():
    c = W.case("quad", seed=3, nx=9, ny=8)
    A = c.vals.copy()
    d0 = int(np.nonzero(c.colidx[c.rowptr[0]:c.rowptr[1]] == 0)[0][0])
    A[d0] = 0.0
    c0 = W.BSRCase(c.n, c.rowptr, c.colidx, A, c.b, c.meta)
    for prec in ("f64", "f32"):
        s = DS(c0, prec)
        s.factor(3, "sync")
        X, D = s.factor_host()
        Xo, Do, fo = oracle.factor_sync(c.n, c.rowptr, c.colidx, A, 3)
        assert fo & oracle.FLAG_MODIFIED
        assert s.flags() & 1
        np.testing.assert_array_equal(D[0], np.eye(4))
        if prec == "f64":
            assert_same_bits(X, Xo, "X")
            assert_same_bits(D, Do, "Dinv")
        else:
            assert rel(X, Xo) <= 1e-5
    A2 = c.vals.copy()
    A2[d0, 1, 2] = np.nan
    s = DS(W.BSRCase(c.n, c.rowptr, c.colidx, A2, c.b, c.meta), "f64")
    s.factor(2, "sync")
    assert s.flags() & 2


def _drop_block(c, i, j):
    """The case without block (i, j) (a structurally non-symmetric pattern)."""
    keep = np.ones(c.nnzb, bool)
    e = c.rowptr[i] + int(np.nonzero(c.colidx[c.rowptr[i]:c.rowptr[i + 1]] == j)[0][0])
    keep[e] = False
    rowptr = np.concatenate([[0], np.cumsum(np.diff(c.rowptr) - (np.arange(c.n) == i))]).astype(np.int32)
    return W.BSRCase(c.n, rowptr, c.colidx[keep], c.vals[keep], c.b, c.meta)


@pytest.mark.parametrize("mode", ["sync", "async"])
@pytest.mark.parametrize("symmetric", [True, False])
def test_first_sweep_flags_every_replaced_initial_inverse(symmetric, mode):
    """The first sweep from A forms the initial inverses inv(A_jj) where the lower blocks need them,
    and a row whose A_ii no other row inverts inverts it itself, so the flag of a replaced initial
    inverse is raised as the oracle (which inverts every diagonal block of X0) raises it: here a
    zero diagonal block on a row that no strictly lower block references (the last row of a chain;
    with the block (3, 2) removed, row 2 of the non-symmetric pattern)."""
    c = W.case("chain", seed=8, n=7)
    row = c.n - 1
    if not symmetric:
        c, row = _drop_block(c, 3, 2), 2
    A = c.vals.copy()
    A[c.rowptr[row] + int(np.nonzero(c.colidx[c.rowptr[row]:c.rowptr[row + 1]] == row)[0][0])] = 0.0
    c0 = W.BSRCase(c.n, c.rowptr, c.colidx, A, c.b, c.meta)
    _, _, fo = oracle.factor_sync(c.n, c.rowptr, c.colidx, A, 1)
    assert fo & oracle.FLAG_MODIFIED
    s = DS(c0, "f64")
    s.factor(1, mode)
    assert s.flags() & 1
    # and none on the unmodified matrix
    s = DS(c, "f64")
    s.factor(1, mode)
    _, _, fo = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 1)
    assert s.flags() == fo == 0


def _lower_pairs_in_one_load_chunk(c, chunk=2):
    """Rows with strictly lower blocks (i, j1), (i, j2) in one load chunk of the sweep (positions
    b0 + 2m, b0 + 2m + 1) where j1 is in the update set of (i, j2), i.e. (j1, j2) is in the
    pattern."""
    S = {(i, int(j)) for i in range(c.n) for j in c.colidx[c.rowptr[i]:c.rowptr[i + 1]]}
    hits = 0
    for i in range(c.n):
        b0 = int(c.rowptr[i])
        low = [int(j) for j in c.colidx[b0:c.rowptr[i + 1]] if j < i]
        for m in range(0, len(low) - 1, chunk):
            hits += (low[m], low[m + 1]) in S
    return hits


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["nine23x17", "random1000"])
def test_first_async_sweep_from_A_ignores_the_output_buffer(name, prec):
    """The first in-place sweep from X0 = A takes U_kj and the inverses inv(A_jj) from A and the
    row's own L_ik from this sweep, each lower block computed after the ones before it in the row:
    it reads nothing of the output buffer before writing it. Its result is therefore the same
    whatever the buffers held (NaN, zero, a huge value), finite, and raises no flag, also where a
    lower block's update set holds the block loaded beside it (nine-point and random patterns)."""
    c = get(name)
    assert _lower_pairs_in_one_load_chunk(c) > 0
    s = DS(c, prec)
    out = []
    for fill in (float("nan"), 0.0, 1e30):
        s.LU.fill_(fill)
        s.Dinv.fill_(fill)
        s.flags(clear=True)
        s.factor(1, "async")
        assert s.flags() == 0, fill
        X, D = s.factor_host()
        assert np.isfinite(X).all() and np.isfinite(D).all(), fill
        out.append((X, D))
    for X, D in out[1:]:
        assert_same_bits(X, out[0][0], "X")
        assert_same_bits(D, out[0][1], "Dinv")


def _factor_apply_solve(s, mode, fill):
    """Factor (2 sweeps from A), one apply (3 sweeps) and one FGMRES solve, every buffer the
    library writes (factor, inverses, workspace, z, x) filled with `fill` bytes beforehand."""
    s.LU.view(torch.uint8).fill_(fill)
    s.Dinv.view(torch.uint8).fill_(fill)
    s.work.fill_(fill)
    s.x.view(torch.uint8).fill_(fill)
    s.flags(clear=True)
    s.factor(2, mode)
    X, D = s.factor_host()
    flags = s.flags(clear=True)
    r = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, 4 * s.n)).cuda()
    z = torch.empty_like(r).view(torch.uint8).fill_(fill).view(torch.float64)
    s.apply(r, z, 3, mode)
    st, res = s.solve(apply_sweeps=3, mode=mode, rtol=1e-6, maxit=200)
    return X, D, flags, z.cpu().numpy(), st, res, s.x.cpu().numpy()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", ["sync", "async", "serial", "chunk_sync", "chunk_async"])
@pytest.mark.parametrize("name", ["nine23x17", "tri40x30_rcm"])
def test_results_do_not_depend_on_prior_buffer_contents(name, mode, prec):
    """Every path reads only what it has written before (or the inputs): with all output and
    workspace bytes set to 0xFF (NaN in either precision) beforehand, the factor, an apply and an
    FGMRES solve stay finite, raise no flag and converge; the deterministic modes give the same
    bits as after zero-filled buffers."""
    c = get(name)
    s = DS(c, prec, restart=30)
    if mode.startswith("chunk"):
        s.set_chunks(8)
    runs = [_factor_apply_solve(s, mode, fill) for fill in (0xFF, 0x00)]
    for X, D, flags, z, st, res, x in runs:
        assert flags == 0
        assert np.isfinite(X).all() and np.isfinite(D).all() and np.isfinite(z).all() and np.isfinite(x).all()
        assert st == 0 and res["converged"]
    if mode in ("sync", "serial", "chunk_sync"):
        for a, b, what in zip(runs[0], runs[1], ("X", "Dinv", "flags", "z", "status", "result", "x")):
            if what in ("X", "Dinv", "z", "x"):
                assert_same_bits(a, b, what)


# ------------------------------------------------------------------ apply sweeps (a5, a6)
@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("nsw", [0, 1, 2, 3, 5])
def test_apply_sync_f64(name, nsw):
    c = get(name)
    s = DS(c, "f64")
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 2)
    s.set_factor(Xo, Do)
    r = np.random.default_rng(nsw).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, nsw, "sync")
    ref = oracle.apply_sync(c.n, c.rowptr, c.colidx, Xo, Do, r, nsw)
    assert_same_bits(zt.cpu().numpy(), ref, "z")


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("nsw", [1, 2, 3])
def test_apply_sync_f32(name, nsw):
    c = get(name)
    s = DS(c, "f32")
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 1)
    X = Xo.astype(np.float32).astype(np.float64)   # the oracle factor as FP32 storage holds it
    D = Do.astype(np.float32).astype(np.float64)
    s.set_factor(X, D)
    r = np.random.default_rng(10 + nsw).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, nsw, "sync")
    e, worst = apply_bars(c, X, D, r, nsw).check(zt.cpu().numpy(), name)
    print(f"{name} f32 apply {nsw}: rel {e:.2e}, worst cell at {worst:.2f} of its bar")


@pytest.mark.parametrize("name", ["quad32", "tri40x30_rcm", "aniso50x20_line", "chain7"])
def test_apply_exact_at_levels(name):
    """Theorem 3 (tight form): once the sweep count reaches the number of levels, sync and
    async sweeps return the exact triangular solves (Algorithm 1)."""
    c = get(name)
    nl, nu, _, _ = oracle.levels(c.n, c.rowptr, c.colidx)
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    r = np.random.default_rng(2).uniform(-1, 1, 4 * c.n)
    ref = oracle.trisolve_exact(c.n, c.rowptr, c.colidx, Xs, Ds, r)
    s = DS(c, "f64")
    s.set_factor(Xs, Ds)
    rt = torch.from_numpy(r).cuda()
    for mode in ("sync", "async"):
        zt = torch.zeros_like(rt)
        s.apply(rt, zt, max(nl, nu), mode)
        # every entry is then computed from final values by the substitution's operations
        assert_same_bits(zt.cpu().numpy(), ref, mode)


def test_apply_async_converges_to_exact():
    c = get("tri40x30_rcm")
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    r = np.random.default_rng(3).uniform(-1, 1, 4 * c.n)
    ref = oracle.trisolve_exact(c.n, c.rowptr, c.colidx, Xs, Ds, r)
    s = DS(c, "f64")
    s.set_factor(Xs, Ds)
    rt = torch.from_numpy(r).cuda()
    errs = []
    for nsw in (1, 2, 4, 8):
        zt = torch.zeros_like(rt)
        s.apply(rt, zt, nsw, "async")
        e_async = rel(zt.cpu().numpy(), ref)
        e_sync = rel(oracle.apply_sync(c.n, c.rowptr, c.colidx, Xs, Ds, r, nsw), ref)
        assert np.isfinite(e_async)
        errs.append((nsw, e_async, e_sync))
    print("nsw, async error, sync error:", errs)
    assert errs[-1][1] < errs[0][1]


# ------------------------------------------------------------------ SpMV (a7)
@pytest.mark.parametrize("name", CASES)
def test_spmv(name):
    c = get(name)
    s = DS(c, "f64")
    x = np.random.default_rng(4).uniform(-1, 1, 4 * c.n)
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    s.spmv(xt, yt)
    ref = oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)
    assert rel(yt.cpu().numpy(), ref) <= 1e-13


# ------------------------------------------------------------------ FGMRES (a8, a9)
@pytest.mark.parametrize("name", ["quad32", "tri40x30_rcm", "nine23x17", "aniso50x20_line"])
def test_fgmres_f64_matches_oracle(name):
    c = get(name)
    s = DS(c, "f64", restart=30)
    s.factor(3, "sync")
    st, res = s.solve(apply_sweeps=3, mode="sync", rtol=1e-6, maxit=300)
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 3)
    ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Xo, Do, restart=30, maxit=300, rtol=1e-6, apply_nsw=3)
    assert st == 0 and res["converged"] and ref["converged"]
    assert abs(res["iters"] - ref["iters"]) <= 1
    assert res["rel_true_residual"] <= 1e-6 and ref["rel_true_residual"] <= 1e-6
    x = s.x.cpu().numpy()
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    assert abs(true - res["rel_true_residual"]) <= 1e-10
    if res["iters"] == ref["iters"]:
        assert rel(x, ref["x"]) <= 1e-10


@pytest.mark.parametrize("apply_sweeps", [2, 4])
@pytest.mark.parametrize("name", ["quad32", "nine23x17"])
def test_fgmres_even_apply_sweeps(name, apply_sweeps):
    """With an even number of apply sweeps the last backward sweep runs its workgroups descending
    and the Arnoldi SpMV ascending (the opposite of 3 sweeps). Same checks as the odd case:
    iteration count within one of the oracle, true residual confirmed by the oracle SpMV, x within
    1e-10 when the counts agree."""
    c = get(name)
    s = DS(c, "f64", restart=30)
    s.factor(3, "sync")
    st, res = s.solve(apply_sweeps=apply_sweeps, mode="sync", rtol=1e-6, maxit=300)
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 3)
    ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Xo, Do, restart=30, maxit=300, rtol=1e-6,
                        apply_nsw=apply_sweeps)
    assert st == 0 and res["converged"] and ref["converged"]
    assert abs(res["iters"] - ref["iters"]) <= 1
    x = s.x.cpu().numpy()
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    assert true <= 1e-6 and abs(true - res["rel_true_residual"]) <= 1e-10
    if res["iters"] == ref["iters"]:
        assert rel(x, ref["x"]) <= 1e-10


def test_fgmres_second_gram_schmidt_pass():
    """A = I + 1e-3 B with the identity preconditioner (no apply sweeps): each new Arnoldi vector
    A v_k lies almost in the span of the basis, so the first classical Gram-Schmidt pass cancels
    nearly all of it and the second pass runs at every step (reorth = iters). The GPU solve must
    still match the oracle's modified Gram-Schmidt FGMRES: same iteration count within one, the
    true residual confirmed by an oracle SpMV, and x within 1e-10 when the counts agree."""
    import dataclasses
    c0 = get("quad32")
    rows = np.repeat(np.arange(c0.n), np.diff(c0.rowptr))
    vals = 1e-3 * c0.vals / np.abs(c0.vals).max()
    vals[rows == c0.colidx] = np.eye(4)
    c = dataclasses.replace(c0, vals=vals)
    s = DS(c, "f64", restart=30)
    for restart in (30, 2):   # 2: restart cycles, each starting from a true residual
        st, res = s.solve(apply_sweeps=0, mode="sync", rtol=1e-12, maxit=200, restart=restart)
        ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, np.zeros((c.nnzb, 4, 4)), np.zeros((c.n, 4, 4)),
                            restart=restart, maxit=200, rtol=1e-12, apply_nsw=0)
        print(f"restart {restart}: gpu iters {res['iters']} reorth {res['reorth']} rel {res['rel_true_residual']:.2e}; "
              f"oracle iters {ref['iters']}")
        assert st == 0 and res["converged"] and ref["converged"]
        assert res["reorth"] == res["iters"] >= 3
        assert abs(res["iters"] - ref["iters"]) <= 1
        x = s.x.cpu().numpy()
        true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
        assert true <= 1e-12 and abs(true - res["rel_true_residual"]) <= 1e-13
        if res["iters"] == ref["iters"]:
            assert rel(x, ref["x"]) <= 1e-10


@pytest.mark.parametrize("name", ["quad32", "tri40x30_rcm", "aniso50x20_line"])
def test_fgmres_f32_sync_preconditioner(name):
    """FP32 factor and sweeps, FP64 Krylov, synchronous sweeps: same outcome as the FP64 oracle
    (both converge within one iteration of each other, or both fail to converge), and the
    double-precision true residual matches an oracle SpMV on the returned x."""
    from paper_1912_00539_amd import abilu as L
    c = get(name)
    s = DS(c, "f32", restart=30)
    s.factor(1, "sync")
    st, res = s.solve(apply_sweeps=3, mode="sync", rtol=1e-2, maxit=300)
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 1)
    ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Xo, Do, restart=30, maxit=300, rtol=1e-2, apply_nsw=3)
    print(f"iters gpu {res['iters']} oracle {ref['iters']}, converged {res['converged']} / {ref['converged']}")
    assert bool(res["converged"]) == ref["converged"]
    if ref["converged"]:
        assert st == 0 and abs(res["iters"] - ref["iters"]) <= 1
    else:
        assert st == L.ABILU_WARN_NOCONV
    x = s.x.cpu().numpy()
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    assert abs(true - res["rel_true_residual"]) <= 1e-10 * max(1.0, true)
    if res["converged"]:
        assert true <= 1e-2


@pytest.mark.parametrize("name", ["quad32", "tri40x30_rcm", "aniso50x20_line"])
def test_fgmres_f32_async_preconditioner(name):
    """Asynchronous factor and sweeps (nondeterministic): the solve converges, its true residual
    is confirmed by an oracle SpMV, and the iteration count is reported beside the oracle's with
    the one-worker (Gauss-Seidel) factor, which is the sequential ILU(0) after one sweep, and with
    the Jacobi-type factor."""
    c = get(name)
    s = DS(c, "f32", restart=30)
    s.factor(1, "async")
    st, res = s.solve(apply_sweeps=3, mode="async", rtol=1e-2, maxit=300)
    Xg, Dg, _ = oracle.factor_gs(c.n, c.rowptr, c.colidx, c.vals, 1)
    gs = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Xg, Dg, restart=30, maxit=300, rtol=1e-2, apply_nsw=3)
    print(f"iters gpu async {res['iters']}, oracle one-worker {gs['iters']}")
    assert st == 0 and res["converged"]
    x = s.x.cpu().numpy()
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    assert true <= 1e-2 and abs(true - res["rel_true_residual"]) <= 1e-10


def test_fgmres_restarts_and_noconv():
    c = W.case("quad", seed=6, nx=30, ny=30, s=0.05)
    s = DS(c, "f64", restart=4)
    s.factor(1, "sync")
    st, res = s.solve(apply_sweeps=1, mode="sync", rtol=1e-8, maxit=400)
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 1)
    ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Xo, Do, restart=4, maxit=400, rtol=1e-8, apply_nsw=1)
    assert res["converged"] and ref["converged"] and res["restarts"] >= 2
    assert abs(res["iters"] - ref["iters"]) <= 1
    from paper_1912_00539_amd import abilu as L
    st, res = s.solve(apply_sweeps=0, mode="sync", rtol=1e-12, maxit=3)
    assert st == L.ABILU_WARN_NOCONV and not res["converged"] and res["iters"] == 3


def test_fgmres_nonzero_initial_guess():
    """x0 given: the solve starts from r0 = b - A x0 (oracle FGMRES from the same x0)."""
    c = get("tri40x30_rcm")
    s = DS(c, "f64", restart=30)
    s.factor(2, "sync")
    x0 = np.random.default_rng(9).uniform(-1, 1, 4 * c.n)
    st, res = s.solve(apply_sweeps=3, mode="sync", rtol=1e-6, maxit=300, x0=torch.from_numpy(x0).cuda())
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 2)
    ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Xo, Do, restart=30, maxit=300, rtol=1e-6, apply_nsw=3,
                        x0=x0)
    assert st == 0 and res["converged"] and abs(res["iters"] - ref["iters"]) <= 1
    if res["iters"] == ref["iters"]:
        assert rel(s.x.cpu().numpy(), ref["x"]) <= 1e-10


def test_fgmres_unpreconditioned_matches_oracle():
    c = W.case("quad", seed=5, nx=12, ny=11, s=0.5)
    s = DS(c, "f64", restart=10)
    st, res = s.solve(apply_sweeps=0, rtol=1e-9, maxit=200)
    Z = np.zeros_like(c.vals); D0 = np.zeros((c.n, 4, 4))
    ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Z, D0, restart=10, maxit=200, rtol=1e-9, apply_nsw=0)
    assert res["converged"] and abs(res["iters"] - ref["iters"]) <= 1


def test_stream_copy():
    from paper_1912_00539_amd import abilu as L
    src = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    L.abilu_stream_copy(dst, src, src.numel() * 8)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_profile_records_launches():
    from paper_1912_00539_amd import abilu as L
    c = get("quad32")
    s = DS(c, "f32")
    L.abilu_profile_enable(True, 1024)
    s.factor(2, "sync")
    rep = L.abilu_profile_report()
    L.abilu_profile_enable(False)
    assert rep["factor_sweep_f32_sync_fromA"][0] == 1 and rep["factor_sweep_f32_sync"][0] == 1


# ------------------------------------------------------------------ full size (4M cells)
@pytest.mark.slow
def test_full_size_tri2000_f32():
    """The benchmark workload at full size, in the benchmark's launch configuration: 1 sync FP32
    factor sweep vs the FP64 oracle, block by block; the FP64 sweep bit for bit; 3 apply sweeps vs
    the oracle on the oracle's factor rounded to FP32 on the host, cell by cell; SpMV bit for bit;
    FGMRES(50) true residual checked by an oracle SpMV on the returned x."""
    c = W.case("tri2000")
    s64 = DS(c, "f64", restart=1)
    s64.factor(1, "sync")
    X, D = s64.factor_host()
    del s64
    bars = F32Bars(c, 1)
    assert_same_bits(X, bars.Xo, "X f64")
    assert_same_bits(D, bars.Do, "Dinv f64")
    s = DS(c, "f32", restart=50)
    s.factor(1, "sync")
    X, D = s.factor_host()
    report("tri2000 f32 1 sweep", bars.check(X, D, "tri2000"))
    Xo = bars.Xo.astype(np.float32).astype(np.float64)   # what the FP32 factor storage holds
    Do = bars.Do.astype(np.float32).astype(np.float64)
    del X, D, bars
    s.set_factor(Xo, Do)
    r = np.random.default_rng(0).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, 3, "sync")
    e, worst = apply_bars(c, Xo, Do, r, 3).check(zt.cpu().numpy(), "tri2000")
    del Xo, Do
    print(f"tri2000 f32 apply 3: rel {e:.2e}, worst cell at {worst:.2f} of its bar")
    s.spmv(rt, zt)
    assert rel(zt.cpu().numpy(), oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, r)) <= 1e-13
    for mode, nsw in (("async", 1), ("sync", 2)):
        s.factor(nsw, mode)
        st, res = s.solve(apply_sweeps=3, mode=mode, rtol=1e-2, maxit=500, restart=50)
        print(mode, nsw, res)
        assert st == 0 and res["converged"]
    x = s.x.cpu().numpy()
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    assert true <= 1e-2 and abs(true - res["rel_true_residual"]) <= 1e-10


@pytest.mark.slow
@pytest.mark.parametrize("cfl", [10.0, 100.0, 1000.0])
def test_full_size_tri300(cfl):
    """The 180,000-triangle workload (300 x 300 split quads, random permutation + RCM) at CFL 10,
    100 and 1000: synchronous FP64 sweeps 1, 2, 4 bit for bit against the oracle; FP32 vs the FP64
    oracle block by block; two apply sweeps bit for bit; FGMRES with the asynchronous FP32
    preconditioner (1 build sweep, 2 apply sweeps) converges, true residual confirmed by the oracle
    SpMV."""
    c = W.case("tri300", cfl=cfl)
    s64 = DS(c, "f64", restart=30)
    for nsw in (1, 2, 4):
        s64.factor(nsw, "sync")
        X, D = s64.factor_host()
        Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, nsw)
        assert_same_bits(X, Xo, f"X {nsw}")
        assert_same_bits(D, Do, f"Dinv {nsw}")
    r = np.random.default_rng(1).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s64.set_factor(Xo, Do)
    s64.apply(rt, zt, 2, "sync")
    assert_same_bits(zt.cpu().numpy(), oracle.apply_sync(c.n, c.rowptr, c.colidx, Xo, Do, r, 2), "z")
    s32 = DS(c, "f32", restart=30)
    s32.factor(2, "sync")
    X32, D32 = s32.factor_host()
    report(f"tri300 CFL {cfl:g} f32 2 sweeps", F32Bars(c, 2).check(X32, D32, f"tri300 {cfl}"))
    s32.factor(1, "async")
    st, res = s32.solve(apply_sweeps=2, mode="async", rtol=1e-2, maxit=300)
    x = s32.x.cpu().numpy()
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    print(f"tri300 CFL {cfl:g}: async FP32 FGMRES iters {res['iters']}, true residual {true:.2e}")
    assert st == 0 and res["converged"] and true <= 1e-2 and abs(true - res["rel_true_residual"]) <= 1e-10


@pytest.mark.slow
def test_full_size_tri300_fgmres_f64_matches_oracle():
    """FGMRES(30) at full size in FP64 to a tight tolerance (1e-8, about ten Arnoldi steps): the
    synchronous two-sweep factor and apply are the oracle's bit for bit, so the GPU's classical
    Gram-Schmidt (twice when needed) and the oracle's modified Gram-Schmidt must reach the same
    iteration count within one, true residuals below rtol on both, and, at equal counts, the same
    x to 1e-10 relative."""
    c = W.case("tri300", cfl=100.0)
    s = DS(c, "f64", restart=30)
    s.factor(2, "sync")
    st, res = s.solve(apply_sweeps=2, mode="sync", rtol=1e-8, maxit=300)
    Xo, Do, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 2)
    ref = oracle.fgmres(c.n, c.rowptr, c.colidx, c.vals, c.b, Xo, Do, restart=30, maxit=300, rtol=1e-8, apply_nsw=2)
    x = s.x.cpu().numpy()
    bn = np.linalg.norm(c.b)
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / bn
    true_ref = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, ref["x"])) / bn
    print(f"tri300 FP64 FGMRES to 1e-8: gpu {res['iters']} iterations ({true:.2e}), oracle {ref['iters']} ({true_ref:.2e})")
    assert st == 0 and res["converged"] and ref["converged"]
    assert abs(res["iters"] - ref["iters"]) <= 1
    assert true <= 1e-8 and true_ref <= 1e-8 and abs(true - res["rel_true_residual"]) <= 1e-12
    if res["iters"] == ref["iters"]:
        assert rel(x, ref["x"]) <= 1e-10


@pytest.mark.slow
@pytest.mark.parametrize("order", ["line", "rcm"])
def test_full_size_aniso1000(order):
    """The 500,000-cell anisotropic workload (1000 x 500, aspect ratio 1000 at the wall) in line
    and RCM order: FP64 synchronous sweeps (1 and 2) bit for bit against the oracle; FP32 block by
    block against the oracle on A and on A rounded to float, the errors stated; FGMRES with the
    asynchronous FP32 preconditioner converges in both orders."""
    c = W.case("aniso1000", order=order)
    for nsw in (1, 2):
        bars = F32Bars(c, nsw)
        s = DS(c, "f64", restart=1)
        s.factor(nsw, "sync")
        X, D = s.factor_host()
        assert_same_bits(X, bars.Xo, f"X f64 {nsw}")
        assert_same_bits(D, bars.Do, f"Dinv f64 {nsw}")
        del s
        s = DS(c, "f32", restart=1)
        s.factor(nsw, "sync")
        X, D = s.factor_host()
        report(f"aniso1000 {order} f32 {nsw} sweeps", bars.check(X, D, f"aniso1000 {order} {nsw}"))
        del s, bars
    s = DS(c, "f32", restart=30)
    s.factor(1, "async")
    st, res = s.solve(apply_sweeps=3, mode="async", rtol=1e-2, maxit=300)
    x = s.x.cpu().numpy()
    true = np.linalg.norm(c.b - oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, x)) / np.linalg.norm(c.b)
    print(f"aniso1000 {order}: async FP32 FGMRES iters {res['iters']}, true residual {true:.2e}")
    assert st == 0 and res["converged"] and true <= 1e-2


# ------------------------------------------------------------------ single-worker schedule (P8)
@pytest.mark.parametrize("name", CASES)
def test_factor_serial_equals_gauss_seidel(name):
    """The asynchronous in-place sweep run by one worker over the rows in order is a Gauss-Seidel
    sweep (oracle_factor_gs); from X0 = A one such sweep is the sequential block ILU(0)
    (Sections 3.3, 4.2). Exercises the in-place reads of fresh L_ik, U_kj and Dinv_j exactly,
    including off-diagonal update sets (nine-point and random patterns)."""
    c = get(name)
    s = DS(c, "f64")
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    for nsw in (1, 2):
        s.factor(nsw, "serial")
        X, D = s.factor_host()
        Xg, Dg, _ = oracle.factor_gs(c.n, c.rowptr, c.colidx, c.vals, nsw)
        assert_same_bits(X, Xg, f"X {nsw}")
        assert_same_bits(D, Dg, f"Dinv {nsw}")
        if nsw == 1:
            assert_same_bits(X, Xs, "X vs sequential ILU(0)")


@pytest.mark.parametrize("name", ["quad32", "tri40x30_rcm", "nine23x17", "random1000", "aniso50x20_line", "chain7"])
def test_apply_serial_is_exact_substitution(name):
    """One forward sweep by one worker in ascending row order is forward substitution, one
    backward sweep in descending order back substitution: z = (LU)^{-1} r (Algorithm 1)."""
    c = get(name)
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    r = np.random.default_rng(5).uniform(-1, 1, 4 * c.n)
    ref = oracle.trisolve_exact(c.n, c.rowptr, c.colidx, Xs, Ds, r)
    s = DS(c, "f64")
    s.set_factor(Xs, Ds)
    rt = torch.from_numpy(r).cuda()
    for nsw in (1, 2):
        zt = torch.zeros_like(rt)
        s.apply(rt, zt, nsw, "serial")
        assert_same_bits(zt.cpu().numpy(), ref, f"z {nsw}")


# ------------------------------------------------------------------ warm start across a Jacobian sequence
@pytest.mark.parametrize("name", ["tri40x30_rcm", "nine23x17", "aniso50x20_line"])
def test_warm_start_sequence_matches_oracle(name):
    """A pseudo-time sequence of drifting Jacobians, each factored by one synchronous sweep
    warm-started from the previous step's factor (the previous factors as the initial guess,
    Section 3.3): the GPU chain equals the oracle's chain, step by step, in FP64."""
    c = get(name)
    s = DS(c, "f64")
    X_or = None
    for t, (vals, b) in enumerate(W.jacobian_sequence(c, W.cfl_ramp(4, 10.0, 2.0), drift=0.01, seed=9)):
        s.load_values(vals, b)
        s.factor(1, "sync", init="A" if t == 0 else "LU")
        X, D = s.factor_host()
        X_or, D_or, _ = oracle.factor_sync(c.n, c.rowptr, c.colidx, vals, 1, X0=X_or)
        assert_same_bits(X, X_or, f"X step {t}")
        assert_same_bits(D, D_or, f"Dinv step {t}")


def test_warm_start_sequence_async_f32():
    """The asynchronous FP32 warm start along the sequence converges FGMRES at every step, with
    true residuals confirmed by the oracle SpMV; its ILU residual is reported beside a cold start
    from A."""
    c = get("tri40x30_rcm")
    warm, cold = DS(c, "f32"), DS(c, "f32")
    out = []
    for t, (vals, b) in enumerate(W.jacobian_sequence(c, W.cfl_ramp(6), drift=0.01, seed=4)):
        for sysm, init in ((warm, "A" if t == 0 else "LU"), (cold, "A")):
            sysm.load_values(vals, b)
            sysm.factor(1, "async", init=init)
        rw, rc = warm.ilu_residual(), cold.ilu_residual()
        st, res = warm.solve(apply_sweeps=3, mode="async", rtol=1e-2, maxit=300)
        x = warm.x.cpu().numpy()
        true = np.linalg.norm(b - oracle.spmv(c.n, c.rowptr, c.colidx, vals, x)) / np.linalg.norm(b)
        assert st == 0 and res["converged"] and true <= 1e-2
        out.append((t, rw, rc, res["iters"]))
    print("step, ILU residual warm, cold, FGMRES iterations:", out)


def test_fgmres_degenerate_right_hand_sides():
    """b = 0: converged at once with x = 0 and no iteration (||b|| = 0 is taken as 1 in the
    tolerance). An initial guess that already solves the system (computed by dense LU on the host):
    the first true residual meets the tolerance and no iteration runs."""
    c = get("quad32")
    s = DS(c, "f64", restart=30)
    s.factor(2, "sync")
    s.b.zero_()
    st, res = s.solve(apply_sweeps=3, mode="sync", rtol=1e-8, maxit=50)
    assert st == 0 and res["converged"] and res["iters"] == 0
    assert float(s.x.abs().max()) == 0.0
    s.b.copy_(torch.from_numpy(c.b))
    xs = np.linalg.solve(c.dense(), c.b)
    st, res = s.solve(apply_sweeps=3, mode="sync", rtol=1e-8, maxit=50, x0=torch.from_numpy(xs).cuda())
    assert st == 0 and res["converged"] and res["iters"] == 0 and res["rel_true_residual"] <= 1e-8
