"""The C-ABI library loads and exports every entry point include/abilu.h declares; argument
checks that run before any device work (no GPU needed)."""
import ctypes as C
import glob
import os
import re

import pytest

from paper_1912_00539_amd import abilu as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("ABILU")))


def test_header_declares_the_boundary():
    assert any(h.endswith("abilu.h") for h in HEADERS)
    names = declared_functions()
    for required in ("abilu_build_pattern", "abilu_factor", "abilu_apply", "abilu_spmv", "fgmres_solve",
                     "abilu_ilu_residual", "abilu_workspace_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    for st in (0, 1, 2, -1, -2, -3, -4, -5):
        s = L.status_string(st)
        assert isinstance(s, str) and len(s) > 0
    assert "invalid argument" in L.status_string(L.ABILU_EINVAL)


def test_argument_checks_without_device():
    lib = L.lib()
    out = C.c_void_p()
    # bad block size / negative size / null output are rejected before any HIP call
    assert lib.abilu_build_pattern(4, None, None, 3, None, C.byref(out)) == L.ABILU_EINVAL
    assert lib.abilu_build_pattern(-1, None, None, 4, None, C.byref(out)) == L.ABILU_EINVAL
    assert lib.abilu_build_pattern(2**31 - 1, None, None, 4, None, C.byref(out)) == L.ABILU_EINVAL
    assert lib.abilu_build_pattern(4, None, None, 4, None, None) == L.ABILU_EINVAL
    assert lib.abilu_workspace_bytes(None, L.ABILU_F32, 30) == 0
    assert lib.abilu_factor(None, None, None, None, L.ABILU_F32, 1, 0, 0, None, 0, None) == L.ABILU_EINVAL
    assert lib.abilu_apply(None, None, None, L.ABILU_F32, None, None, 1, 0, None, 0, None) == L.ABILU_EINVAL
    assert lib.abilu_spmv(None, None, None, None, None) == L.ABILU_EINVAL
    res = L.FgmresResult()
    assert lib.fgmres_solve(None, None, None, None, 30, 10, 1e-2, None, None, 0, 3, 0, 0, None, 0, None,
                            C.byref(res)) == L.ABILU_EINVAL
    assert lib.abilu_pattern_set_chunks(None, 64, 0, None) == L.ABILU_EINVAL
    assert lib.abilu_pattern_chunk_info(None, None, None, None, None, None, None, None) == L.ABILU_EINVAL
    assert lib.abilu_pattern_chunk_export(None, 0, None, None, None, None) == L.ABILU_EINVAL
    assert lib.abilu_stream_copy(None, None, 7, None) == L.ABILU_EINVAL
    assert lib.abilu_pattern_info(None, None, None, None, None, None, None) == L.ABILU_EINVAL
    assert lib.abilu_pattern_depth(None, None, None, None, None, None, None, None) == L.ABILU_EINVAL
    d = C.c_double()
    assert lib.abilu_factor_maxdiff(None, L.ABILU_F32, None, None, None, 0, C.byref(d), C.byref(d), None) == L.ABILU_EINVAL
    assert lib.abilu_jacobi_norms(None, L.ABILU_F32, None, None, None, 0, C.byref(d), C.byref(d), None) == L.ABILU_EINVAL
    assert lib.abilu_profile_enable(1, 0) == L.ABILU_EINVAL


def test_gen_sizes_match_host_generator():
    """abilu_gen_sizes (host arithmetic only) gives the host twin's N and Z."""
    from paper_1912_00539_amd import workloads as W
    for req in (dict(kind="tri", nx=7, ny=5, cfl=50.0, seed=3), dict(kind="aniso", nx=9, ny=4, cfl=10.0, seed=4),
                dict(kind="tri", nx=1, ny=1, cfl=1.0, seed=0), dict(kind="aniso", nx=1, ny=3, cfl=1.0, seed=0)):
        c = W.request_case(req)
        assert L.abilu_gen_sizes(req) == (c.n, c.nnzb)
        assert L.abilu_gen_scratch_bytes(req) >= 8 * (c.n + 1) + 16   # row lengths, tile sums and total


def test_gen_rejects_bad_specs():
    for bad in (dict(kind="tri", nx=0, ny=5, cfl=1.0, seed=0), dict(kind="aniso", nx=3, ny=-1, cfl=1.0, seed=0),
                dict(kind="tri", nx=3, ny=3, cfl=0.0, seed=0), dict(kind="tri", nx=3, ny=3, cfl=float("nan"), seed=0),
                dict(kind="tri", nx=40000, ny=40000, cfl=1.0, seed=0)):
        with pytest.raises(L.AbiluError):
            L.abilu_gen_sizes(bad)
        assert L.abilu_gen_scratch_bytes(bad) == 0
    spec = L.GenSpec(7, 3, 3, 1.0, 0)
    assert L.lib().abilu_gen_sizes(C.byref(spec), None, None) == L.ABILU_EINVAL
    assert L.lib().abilu_gen_build(None, None, None, None, None, None, None) == L.ABILU_EINVAL


def test_serve_footprint_host_only():
    """Pool bytes per request (no device work): about 3 kB per cell for an FP32 preconditioner,
    an FP64 system and FGMRES(30) bases; FP64 factors, SYNC ping-pong buffers and longer
    restarts cost more."""
    req = dict(kind="tri", nx=224, ny=224, cfl=100.0, seed=1)
    n, _ = L.abilu_gen_sizes(req)
    base = L.abilu_serve_footprint(L.serve_config(), req)
    assert 2.8e3 <= base / n <= 3.2e3
    assert L.abilu_serve_footprint(L.serve_config(prec="f64"), req) > base
    assert L.abilu_serve_footprint(L.serve_config(mode="sync", factor_sweeps=2), req) > base
    assert L.abilu_serve_footprint(L.serve_config(restart=50), req) > base
    assert L.abilu_serve_footprint(L.serve_config(restart=0), req) == 0
    assert L.abilu_serve_footprint(L.serve_config(restart=257), req) == 0
    assert L.abilu_serve_footprint(L.serve_config(max_active=0), req) == 0
    assert L.abilu_serve_footprint(L.serve_config(), dict(kind="tri", nx=0, ny=1, cfl=1.0, seed=0)) == 0


def test_serve_rejects_bad_arguments():
    lib = L.lib()
    out = C.c_void_p(1)
    cfg = L.serve_config()
    assert lib.abilu_serve_create(C.byref(cfg), None, 1 << 20, C.byref(out)) == L.ABILU_EINVAL
    assert out.value is None
    assert lib.abilu_serve_create(C.byref(cfg), C.c_void_p(4096 + 8), 1 << 20, C.byref(out)) == L.ABILU_EINVAL
    bad = L.serve_config(prec="f32", maxit=-1)
    assert lib.abilu_serve_create(C.byref(bad), C.c_void_p(4096), 1 << 20, C.byref(out)) == L.ABILU_EINVAL
    assert lib.abilu_serve_create(C.byref(cfg), C.c_void_p(4096), 1 << 20, None) == L.ABILU_EINVAL
    assert lib.abilu_serve_destroy(None) == L.ABILU_EINVAL
    assert lib.abilu_serve_step(None, None, None, None) == L.ABILU_EINVAL
    assert lib.abilu_serve_submit(None, None, None) == L.ABILU_EINVAL
    done = C.c_int32()
    assert lib.abilu_serve_poll(None, 0, C.byref(done), None) == L.ABILU_EINVAL
    assert lib.abilu_serve_run(None, None, 0, None, None, None) == L.ABILU_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback: without the built HIP library every entry point raises."""
    import pytest
    from paper_1912_00539_amd import abilu
    monkeypatch.setattr(abilu, "_lib", None)
    monkeypatch.setattr(abilu, "LIB_PATH", "/nonexistent/libabilu.so")
    with pytest.raises(RuntimeError, match="not built"):
        abilu.lib()
