"""abilu_apply_noalloc (the allocation-free preconditioner application) against abilu_apply, through
the C ABI: the same bits in every deterministic mode, on two calls in a row, the second with a
smaller pattern than the first (the device array keeps the first call's contents); patterns beyond
the array's size are refused before anything is launched."""
import numpy as np
import pytest

from paper_1912_00539_amd import workloads as W

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


def _system(case, prec, R=None):
    from paper_1912_00539_amd.runtime import DeviceSystem
    s = DeviceSystem(case, prec=prec, restart=0)
    if R:
        s.set_chunks(R)
    s.factor(2, "sync")
    return s


def _both(s, prec, r, nsw, mode):
    """z from abilu_apply (caller workspace) and from abilu_apply_noalloc."""
    from paper_1912_00539_amd import abilu as L
    z_ref = torch.full_like(r, np.nan)
    z_new = torch.full_like(r, np.nan)
    L.abilu_apply(s.pattern, s.LU, s.Dinv, prec, r, z_ref, nsw, mode, s.work)
    L.abilu_apply_noalloc(s.pattern, s.LU, s.Dinv, prec, r, z_new, nsw, mode)
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_new.cpu().numpy()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode,nsw", [("sync", 3), ("sync", 2), ("sync", 1), ("sync", 0), ("serial", 1),
                                      ("chunk_sync", 2)])
def test_noalloc_equals_apply_two_calls(prec, mode, nsw):
    big = W.case("tri", seed=21, nx=70, ny=60, order="rcm", shift="cfl", cfl=100.0)     # 8,400 cells
    small = W.case("quad32")                                                             # 1,024 cells
    for c in (big, small):
        s = _system(c, prec, R=64 if mode.startswith("chunk") else None)
        r = torch.from_numpy(np.random.default_rng(c.n).uniform(-1, 1, 4 * c.n)).cuda()
        ref, new = _both(s, prec, r, nsw, mode)
        assert np.isfinite(ref).all()
        np.testing.assert_array_equal(new, ref)


def test_noalloc_async_is_exact_at_levels():
    """The in-place mode (nondeterministic in general) gives the exact substitution once the sweep
    count reaches the level count, for both entry points alike."""
    import oracle
    c = W.case("tri", seed=22, nx=12, ny=9, order="rcm", shift="cfl", cfl=100.0)
    s = _system(c, "f64")
    nl, nu, _, _ = oracle.levels(c.n, c.rowptr, c.colidx)
    r = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, 4 * c.n)).cuda()
    ref, new = _both(s, "f64", r, max(nl, nu), "async")
    np.testing.assert_array_equal(new, ref)


def chain_pattern(n):
    """Block tridiagonal pattern: row i holds columns i-1, i, i+1 (those in range)."""
    deg = np.full(n, 3, np.int64)
    deg[0] = deg[-1] = 2
    rowptr = np.zeros(n + 1, np.int64)
    rowptr[1:] = np.cumsum(deg)
    offs = np.concatenate([[0, 1], np.tile([-1, 0, 1], n - 2), [-1, 0]])
    return rowptr, np.repeat(np.arange(n), deg) + offs


@pytest.mark.parametrize("prec,nmax", [("f32", 1 << 20), ("f64", 1 << 19)])
def test_noalloc_rejects_patterns_beyond_its_array(prec, nmax):
    """N = nmax fits exactly (4 vectors of 4N values fill ABILU_NOALLOC_SCRATCH_BYTES); N = nmax + 1
    is refused with ABILU_EINVAL and an explanation, and z is left untouched."""
    from paper_1912_00539_amd import abilu as L
    for n, ok in ((nmax, True), (nmax + 1, False)):
        rowptr, colidx = chain_pattern(n)
        p = L.abilu_build_pattern(n, torch.from_numpy(rowptr.astype(np.int32)).cuda(),
                                  torch.from_numpy(colidx.astype(np.int32)).cuda())
        dt = torch.float32 if prec == "f32" else torch.float64
        Z = int(rowptr[-1])
        LU = torch.zeros(Z * 16, dtype=dt, device="cuda")
        D = torch.zeros(n * 16, dtype=dt, device="cuda")
        D.view(n, 16)[:, ::5] = 1.0                     # Dinv = I, L = U = 0: z = r
        r = torch.ones(4 * n, dtype=torch.float64, device="cuda")
        z = torch.full_like(r, 7.0)
        if ok:
            L.abilu_apply_noalloc(p, LU, D, prec, r, z, 2, "sync")
            torch.cuda.synchronize()
            assert bool((z == 1.0).all())
        else:
            with pytest.raises(L.AbiluError) as ei:
                L.abilu_apply_noalloc(p, LU, D, prec, r, z, 2, "sync")
            assert ei.value.status == L.ABILU_EINVAL
            assert "ABILU_NOALLOC_SCRATCH_BYTES" in L.abilu_last_error()
            torch.cuda.synchronize()
            assert bool((z == 7.0).all())
        del p
