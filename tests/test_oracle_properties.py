"""Property-based pins of the CPU oracle on random sparse patterns (no GPU).

Random symmetric patterns of 1 to 24 cells, from empty to dense, in random or natural order, with
the seeded finite-volume values. Update sets K(i,j) with common neighbours, long dependency
chains and rows without neighbours all occur. On every drawn case the oracle must satisfy what
the method fixes independently of it:
  - P1: (LU)_ij = A_ij on the pattern, from dense NumPy products (equation bilu);
  - P2: the forward substitution equals right-looking block elimination with dropping;
  - P3: synchronous sweeps reach the sequential factor after D sweeps, D the dependency depth
    (Lemma 2, Theorem 8);
  - P6: one in-place row-major sweep is the sequential factor (Section 3.3);
  - the composite apply with sweep counts at the level counts equals the dense solve with L U
    (Theorem 3).
"""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
from paper_1912_00539_amd import workloads as W  # noqa: E402
from tests.dense_ref import block_ilu0_kij, factors_dense, pattern_mask, rel, to_dense  # noqa: E402

pytestmark = pytest.mark.filterwarnings("ignore")

cases = st.builds(
    lambda n, deg, seed, order: (n, deg, seed, order, W.case("random", seed=seed, n=n, deg=deg, order=order)),
    n=st.integers(1, 24),
    deg=st.sampled_from([0.0, 1.0, 2.5, 4.0, 8.0, 30.0]),
    seed=st.integers(0, 2**31 - 1),
    order=st.sampled_from(["natural", "random"]),
)


@settings(max_examples=300, deadline=None)
@given(cases)
def test_random_patterns_satisfy_the_pins(drawn):
    n, deg, seed, order, c = drawn
    A = to_dense(c.n, c.rowptr, c.colidx, c.vals)
    scale = np.abs(A).max()
    mask = np.kron(pattern_mask(c.n, c.rowptr, c.colidx), np.ones((4, 4), bool))
    X, Dv, flags = oracle.ilu0_seq(c.n, c.rowptr, c.colidx, c.vals)
    assert flags == 0
    # P1
    L, U = factors_dense(c.n, c.rowptr, c.colidx, X)
    assert np.abs(L @ U - A)[mask].max() <= 1e-13 * scale
    for i in range(c.n):
        np.testing.assert_allclose(Dv[i] @ U[4 * i:4 * i + 4, 4 * i:4 * i + 4], np.eye(4), atol=1e-13)
    # P2
    assert rel(X, block_ilu0_kij(c.n, c.rowptr, c.colidx, c.vals)) < 1e-13
    # P3: exact after D sweeps (at least one sweep)
    D, _ = oracle.depth(c.n, c.rowptr, c.colidx)
    Xs, Ds, fs = oracle.factor_sync(c.n, c.rowptr, c.colidx, c.vals, max(D, 1))
    assert fs == 0 and rel(Xs, X) <= 1e-14 and rel(Ds, Dv) <= 1e-14
    # P6
    Xg, Dg, _ = oracle.factor_gs(c.n, c.rowptr, c.colidx, c.vals, 1)
    assert rel(Xg, X) <= 1e-15 and rel(Dg, Dv) <= 1e-15
    # Theorem 3: enough Jacobi sweeps on each factor give the exact preconditioner solve
    nl, nu, _, _ = oracle.levels(c.n, c.rowptr, c.colidx)
    z = oracle.apply_sync(c.n, c.rowptr, c.colidx, X, Dv, c.b, max(nl, nu))
    assert rel(z, np.linalg.solve(L @ U, c.b)) < 1e-11
