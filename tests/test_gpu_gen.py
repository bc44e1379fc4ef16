"""The device request generator (include/abilu_gen.h) against its host twin
(workloads.request_case): the block pattern bit-exact, the values equal up to the summation order
of the diagonal shift (and the last bit of pow() in the anisotropic face scaling)."""
import numpy as np
import pytest

from paper_1912_00539_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REQS = [
    dict(kind="tri", nx=1, ny=1, cfl=10.0, seed=1),
    dict(kind="tri", nx=37, ny=23, cfl=100.0, seed=2),
    dict(kind="tri", nx=64, ny=130, cfl=999.0, seed=3),
    dict(kind="aniso", nx=1, ny=1, cfl=10.0, seed=4),
    dict(kind="aniso", nx=1, ny=7, cfl=10.0, seed=5),
    dict(kind="aniso", nx=45, ny=31, cfl=500.0, seed=6),
    dict(kind="aniso", nx=300, ny=2, cfl=20.0, seed=7),
]


def generate(req):
    from paper_1912_00539_amd import abilu as L
    n, z = L.abilu_gen_sizes(req)
    dev = torch.device("cuda:0")
    rowptr = torch.full((n + 1,), -7, dtype=torch.int32, device=dev)
    colidx = torch.full((z,), -7, dtype=torch.int32, device=dev)
    A = torch.full((z * 16,), float("nan"), dtype=torch.float64, device=dev)
    b = torch.full((4 * n,), float("nan"), dtype=torch.float64, device=dev)
    scratch = torch.empty(L.abilu_gen_scratch_bytes(req), dtype=torch.uint8, device=dev)
    L.abilu_gen_build(req, rowptr, colidx, A, b, scratch)
    torch.cuda.synchronize()
    return n, z, rowptr.cpu().numpy(), colidx.cpu().numpy(), A.cpu().numpy().reshape(z, 4, 4), b.cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("req", REQS, ids=lambda r: f"{r['kind']}{r['nx']}x{r['ny']}")
def test_generator_matches_host_twin(req):
    c = W.request_case(req)
    n, z, rowptr, colidx, A, b = generate(req)
    assert (n, z) == (c.n, c.nnzb)
    np.testing.assert_array_equal(rowptr, c.rowptr)
    np.testing.assert_array_equal(colidx, c.colidx)
    np.testing.assert_array_equal(b, c.b)
    diag = np.zeros(z, bool)
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            diag[e] = colidx[e] == i
    off = ~diag
    # off-diagonal blocks: same operations in the same order (tri: bit-exact; aniso: pow() ulp)
    tol_off = 0.0 if req["kind"] == "tri" else 4e-16
    err = np.abs(A[off] - c.vals[off]).max(initial=0.0) / max(np.abs(c.vals[off]).max(initial=1.0), 1e-300)
    assert err <= tol_off, err
    # diagonal blocks: shift summed over neighbours in another order
    errd = np.abs(A[diag] - c.vals[diag]).max() / np.abs(c.vals[diag]).max()
    assert errd <= 1e-14, errd


def test_generator_serving_size_sample():
    """One request at the serving mix's upper size: pattern exact, values to 1e-14 on sampled rows."""
    req = dict(kind="aniso", nx=1414, ny=707, cfl=300.0, seed=11)
    c = W.request_case(req)
    n, z, rowptr, colidx, A, b = generate(req)
    np.testing.assert_array_equal(rowptr, c.rowptr)
    np.testing.assert_array_equal(colidx, c.colidx)
    np.testing.assert_array_equal(b, c.b)
    rel = np.abs(A - c.vals).max() / np.abs(c.vals).max()
    assert rel <= 1e-14, rel
