"""GPU parity with the CPU oracle on seeded random sparse patterns.

Random symmetric patterns (block diagonal to dense-ish rows), in natural or random order, at
sizes around the 64-row workgroup tile (one row, a ragged tail, several tiles). On each:
  - pattern analysis bit-exact (diagonal positions, update-set pairs);
  - two synchronous FP64 factor sweeps equal the oracle's bit for bit;
  - synchronous sweeps at the dependency depth D equal the sequential factor bit for bit
    (Theorem 8), and in-place asynchronous sweeps reach the same floating-point result;
  - three synchronous FP64 apply sweep pairs equal the oracle's bit for bit, the SpMV within 1e-13
    (its products are summed per block, fused, before the accumulator: rounding order only).
"""
import numpy as np
import pytest

import oracle
from paper_1912_00539_amd import workloads as W
from tests.dense_ref import assert_same_bits, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (cells, mean neighbours, order, seed)
PATTERNS = [
    (1, 0.0, "natural", 101),
    (2, 1.0, "natural", 102),
    (63, 0.0, "random", 103),
    (64, 3.0, "random", 104),
    (65, 6.0, "natural", 105),
    (130, 12.0, "random", 106),
    (257, 2.0, "random", 107),
    (600, 5.0, "natural", 108),
    (1000, 8.0, "random", 109),
    (2049, 4.0, "random", 110),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_00539_amd import abilu
    abilu.lib()
    yield
    torch.cuda.synchronize()


def DS(case, prec="f64"):
    from paper_1912_00539_amd.runtime import DeviceSystem
    return DeviceSystem(case, prec=prec, restart=10)


@pytest.mark.parametrize("n,deg,order,seed", PATTERNS, ids=lambda v: str(v))
def test_random_pattern_parity(n, deg, order, seed):
    from paper_1912_00539_amd import abilu as L
    c = W.case("random", seed=seed, n=n, deg=deg, order=order)
    print(f"random pattern n={n} deg={deg} order={order} seed={seed}: Z={c.nnzb}", flush=True)
    # pattern analysis
    s = DS(c)
    nn, z, npairs = s.pattern.info()
    ptr, pik, pkj = oracle.pairs(c.n, c.rowptr, c.colidx)
    assert (nn, z, npairs) == (c.n, c.nnzb, int(ptr[-1]))
    dp = torch.zeros(max(c.n, 1), dtype=torch.int32, device="cuda")
    pp = torch.zeros(z + 1, dtype=torch.int32, device="cuda")
    a = torch.zeros(max(npairs, 1), dtype=torch.int32, device="cuda")
    b = torch.zeros(max(npairs, 1), dtype=torch.int32, device="cuda")
    L.abilu_pattern_export(s.pattern, dp, pp, a, b)
    torch.cuda.synchronize()
    diag = np.array([c.rowptr[i] + np.nonzero(c.colidx[c.rowptr[i]:c.rowptr[i + 1]] == i)[0][0]
                     for i in range(c.n)])
    np.testing.assert_array_equal(dp.cpu().numpy()[: c.n], diag)
    np.testing.assert_array_equal(pp.cpu().numpy(), ptr)
    np.testing.assert_array_equal(a.cpu().numpy()[:npairs], pik)
    np.testing.assert_array_equal(b.cpu().numpy()[:npairs], pkj)
    # two synchronous sweeps
    s.factor(2, "sync")
    X2, D2 = s.factor_host()
    Xo, Do, fo = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, 2)
    assert_same_bits(X2, Xo, "X")
    assert_same_bits(D2, Do, "Dinv")
    assert s.flags() == fo == 0
    # exactness at the depth, synchronous and asynchronous
    D, _ = oracle.depth(c.n, c.rowptr, c.colidx)
    Xs, Ds, _ = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    s.factor(D, "sync")
    Xg, Dg = s.factor_host()
    assert_same_bits(Xg, Xs, "X at depth")
    assert_same_bits(Dg, Ds, "Dinv at depth")
    t = DS(c)
    t.factor(D + 2, "async")
    Xa, Da = t.factor_host()
    np.testing.assert_array_equal(Xa, Xg)
    np.testing.assert_array_equal(Da, Dg)
    # apply sweeps and SpMV
    s.set_factor(Xo, Do)
    r = np.random.default_rng(seed).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, 3, "sync")
    assert_same_bits(zt.cpu().numpy(), oracle.apply_sync(c.n, c.rowptr, c.colidx, Xo, Do, r, 3), "z")
    yt = torch.zeros_like(rt)
    s.spmv(rt, yt)
    assert rel(yt.cpu().numpy(), oracle.spmv(c.n, c.rowptr, c.colidx, c.vals, r)) <= 1e-13


@pytest.mark.parametrize("runner", ["levels", "rows"])
@pytest.mark.parametrize("R", [3, 16])
@pytest.mark.parametrize("n,deg,order,seed", PATTERNS, ids=lambda v: str(v))
def test_random_pattern_chunked_parity(n, deg, order, seed, R, runner):
    """Chunked synchronous sweeps (Gauss-Seidel within chunks of R consecutive rows, other chunks
    read from the previous sweep, Section 3.3): two factor sweeps and two apply sweep pairs in
    FP64 within 1e-12 of the oracle's chunked iteration, with both chunk runners."""
    from paper_1912_00539_amd.runtime import DeviceSystem
    c = W.case("random", seed=seed, n=n, deg=deg, order=order)
    print(f"random pattern n={n} deg={deg} order={order} seed={seed} R={R} runner={runner}", flush=True)
    s = DeviceSystem(c, prec="f64", restart=10)
    s.set_chunks(R, runner)
    s.factor(2, "chunk_sync")
    X, D = s.factor_host()
    Xo, Do, fo = oracle.factor_chunked(c.n, c.rowptr, c.colidx, c.vals, 2, R)
    assert_same_bits(X, Xo, "X")
    assert_same_bits(D, Do, "Dinv")
    assert s.flags() == fo == 0
    s.set_factor(Xo, Do)
    r = np.random.default_rng(seed + 1).uniform(-1, 1, 4 * c.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    s.apply(rt, zt, 2, "chunk_sync")
    assert_same_bits(zt.cpu().numpy(), oracle.apply_chunked(c.n, c.rowptr, c.colidx, Xo, Do, r, 2, R), "z")
