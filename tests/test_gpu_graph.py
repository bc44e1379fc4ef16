"""The factor and apply entry points only launch kernels on the caller's stream (no allocation, no
memset, no host synchronisation), so a caller can capture them into a HIP graph and replay it. Each
replay must give the bits of the eager calls, with the program's own eager work and
synchronisations between replays (the buffers are overwritten with NaN before every replay)."""
import numpy as np
import pytest

from paper_1912_00539_amd import workloads as W
from tests.dense_ref import assert_same_bits

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


CASES = {
    "nine23x17": lambda: W.case("nine", seed=4, nx=23, ny=17),
    "tri40x30_rcm": lambda: W.case("tri", seed=3, nx=40, ny=30, order="rcm", shift="cfl", cfl=100.0),
}


def _capture(fn):
    """fn() run once on a side stream, then captured into a graph (torch's capture stream)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", ["sync", "serial", "chunk_sync"])
@pytest.mark.parametrize("name", list(CASES))
def test_factor_and_apply_replay_as_a_graph(name, mode, prec):
    from paper_1912_00539_amd.runtime import DeviceSystem
    c = CASES[name]()
    s = DeviceSystem(c, prec=prec, restart=1)
    if mode == "chunk_sync":
        s.set_chunks(8)
    r = torch.from_numpy(np.random.default_rng(11).uniform(-1, 1, 4 * c.n)).cuda()
    z = torch.zeros_like(r)

    def work():
        s.factor(2, mode)
        s.apply(r, z, 3, mode)

    work()
    torch.cuda.synchronize()
    X0, D0 = s.factor_host()
    z0 = z.cpu().numpy()
    g = _capture(work)
    for rep in range(3):
        s.LU.fill_(float("nan"))
        s.Dinv.fill_(float("nan"))
        z.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        X, D = s.factor_host()
        assert_same_bits(X, X0, f"X, replay {rep}")
        assert_same_bits(D, D0, f"Dinv, replay {rep}")
        assert_same_bits(z.cpu().numpy(), z0, f"z, replay {rep}")
        assert s.flags() == 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_apply_replays_as_a_graph(prec):
    """The allocation-free application, the entry point for callers that capture graphs: replays
    equal the workspace form's eager result."""
    from paper_1912_00539_amd import abilu as L
    from paper_1912_00539_amd.runtime import DeviceSystem
    c = CASES["tri40x30_rcm"]()
    s = DeviceSystem(c, prec=prec, restart=0)
    s.factor(2, "sync")
    r = torch.from_numpy(np.random.default_rng(12).uniform(-1, 1, 4 * c.n)).cuda()
    z_ref = torch.zeros_like(r)
    L.abilu_apply(s.pattern, s.LU, s.Dinv, prec, r, z_ref, 3, "sync", s.work)
    z = torch.zeros_like(r)
    g = _capture(lambda: L.abilu_apply_noalloc(s.pattern, s.LU, s.Dinv, prec, r, z, 3, "sync"))
    ref = z_ref.cpu().numpy()
    for rep in range(3):
        z.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_same_bits(z.cpu().numpy(), ref, f"z, replay {rep}")
