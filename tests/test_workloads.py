"""The input generators hold no method arithmetic; these check that the pseudo-time Jacobian
sequence is what its definition says (CPU)."""
import numpy as np

from paper_1912_00539_amd import workloads as W


def _block_1norm(b):
    return max(np.abs(b[:, c]).sum() for c in range(4))


def test_cfl_ramp():
    r = W.cfl_ramp(12, 10.0, 1.5, 1000.0)
    assert r[0] == 10.0 and np.all(np.diff(r) >= 0) and r.max() <= 1000.0
    assert np.allclose(r[1:6] / r[:5], 1.5)


def test_jacobian_sequence_definition():
    c = W.case("tri", seed=3, nx=6, ny=5, order="rcm", shift="cfl", cfl=10.0)
    cfls = W.cfl_ramp(4)
    seq = list(W.jacobian_sequence(c, cfls, drift=0.02, seed=5))
    assert len(seq) == 4
    np.testing.assert_array_equal(seq[0][0], c.vals)       # step 0 is the case itself (same CFL)
    prev = c.vals
    for t, (v, b) in enumerate(seq):
        assert v.shape == c.vals.shape and b.shape == c.b.shape
        assert np.all(np.abs(b / c.b - 1.0) <= 0.02 + 1e-15)
        for i in range(c.n):
            lo, hi = c.rowptr[i], c.rowptr[i + 1]
            cols = c.colidx[lo:hi]
            offs = [e for e in range(lo, hi) if cols[e - lo] != i]
            d = lo + int(np.nonzero(cols == i)[0][0])
            for e in offs:                                  # off-diagonal drift within the bound
                if t > 0:
                    ratio = v[e] / prev[e]
                    assert np.all(np.abs(ratio - 1.0) <= 0.02 + 1e-12)
            ct = sum(_block_1norm(v[e]) for e in offs) * (1.0 + 1.0 / cfls[t])
            c0 = sum(_block_1norm(c.vals[e]) for e in offs) * (1.0 + 1.0 / 10.0)
            np.testing.assert_allclose(v[d] - c.vals[d], (ct - c0) * np.eye(4), atol=1e-12 * max(1.0, ct))
        prev = v
