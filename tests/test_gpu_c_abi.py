"""The C ABI used by a C program alone (tests/c_abi/solve.c, built by __graft_entry__.build()
next to libabilu.so): no Python binding and no torch in that process. The program builds a seeded
2-D block system, factors it (one asynchronous FP32 sweep), solves it with FGMRES(30) to 1e-8 and
checks the returned x against its own host-side residual; it also checks that a bad argument comes
back as ABILU_EINVAL. Run as a child process."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "paper_1912_00539_amd", "lib", "abilu_c_solve")


@pytest.mark.parametrize("nx,ny", [(40, 30), (7, 3), (1, 1)])
def test_c_program_solves(nx, ny):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(BIN):
        pytest.fail("abilu_c_solve is not built: run __graft_entry__.build()")
    out = subprocess.run([BIN, str(nx), str(ny)], capture_output=True, text=True, timeout=120)
    print(out.stdout, out.stderr)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    assert out.stdout.startswith("OK: n=%d " % (nx * ny))
