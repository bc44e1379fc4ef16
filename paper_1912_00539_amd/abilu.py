"""Thin ctypes binding of libabilu.so (include/abilu.h): same entry-point names, argument
marshalling only. Device buffers are torch tensors on the current HIP device; every call is
ordered on torch's current stream unless a stream is given. Every computation runs in the HIP
library: if the library is not built this module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libabilu.so")

ABILU_OK, ABILU_WARN_MODIFIED, ABILU_WARN_NOCONV = 0, 1, 2
ABILU_EINVAL, ABILU_EPATTERN, ABILU_ENOMEM, ABILU_EDEVICE, ABILU_ENONFINITE = -1, -2, -3, -4, -5
ABILU_SYNC, ABILU_ASYNC, ABILU_ASYNC_SERIAL, ABILU_CHUNK_SYNC, ABILU_CHUNK_ASYNC = 0, 1, 2, 3, 4
ABILU_F64, ABILU_F32 = 0, 1
ABILU_INIT_FROM_A, ABILU_INIT_FROM_LU = 0, 1
ABILU_FLAG_MODIFIED, ABILU_FLAG_NONFINITE = 1, 2
ABILU_FGMRES_ZERO_GUESS = 1

MODES = {"sync": ABILU_SYNC, "async": ABILU_ASYNC, "serial": ABILU_ASYNC_SERIAL, "chunk_sync": ABILU_CHUNK_SYNC,
         "chunk_async": ABILU_CHUNK_ASYNC}
PRECS = {"f64": ABILU_F64, "f32": ABILU_F32}
ABILU_CHUNK_AUTO, ABILU_CHUNK_BY_LEVELS, ABILU_CHUNK_BY_ROWS = 0, 1, 2
CHUNK_RUNNERS = {"auto": ABILU_CHUNK_AUTO, "levels": ABILU_CHUNK_BY_LEVELS, "rows": ABILU_CHUNK_BY_ROWS}
INITS = {"A": ABILU_INIT_FROM_A, "LU": ABILU_INIT_FROM_LU}


class AbiluError(RuntimeError):
    def __init__(self, status: int, where: str):
        detail = f" [{abilu_last_error()}]" if status == ABILU_EDEVICE else ""
        super().__init__(f"{where}: {status_string(status)} ({status}){detail}")
        self.status = status


class FgmresResult(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("flags", C.c_uint32), ("reorth", C.c_int32), ("rel_true_residual", C.c_double),
                ("rel_estimate", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class GenSpec(C.Structure):
    """abilu_gen_spec (include/abilu_gen.h)."""
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("cfl", C.c_double),
                ("seed", C.c_uint64)]


GEN_KINDS = {"tri": 0, "aniso": 1}


def gen_spec(req: dict) -> GenSpec:
    return GenSpec(GEN_KINDS[req["kind"]], int(req["nx"]), int(req["ny"]), float(req["cfl"]), int(req["seed"]))


class ServeConfig(C.Structure):
    """abilu_serve_config (include/abilu_serve.h)."""
    _fields_ = [("prec", C.c_int32), ("mode", C.c_int32), ("factor_sweeps", C.c_int32), ("apply_sweeps", C.c_int32),
                ("restart", C.c_int32), ("maxit", C.c_int32), ("rtol", C.c_double), ("max_active", C.c_int32),
                ("reserved", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("gen", GenSpec), ("arrival_s", C.c_double), ("d_x_out", C.c_void_p)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("n", C.c_int32), ("nnzb", C.c_int64), ("iters", C.c_int32),
                ("restarts", C.c_int32), ("converged", C.c_int32), ("reorth", C.c_int32), ("flags", C.c_uint32),
                ("reserved", C.c_int32), ("rel_true_residual", C.c_double), ("t_arrival", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("footprint_bytes", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class ServeStats(C.Structure):
    _fields_ = [("ticks", C.c_int64), ("launches", C.c_int64), ("admitted", C.c_int64), ("retired", C.c_int64),
                ("bytes", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def serve_config(prec: str = "f32", mode: str = "async", factor_sweeps: int = 1, apply_sweeps: int = 3,
                 restart: int = 30, maxit: int = 300, rtol: float = 1e-2, max_active: int = 64) -> ServeConfig:
    return ServeConfig(PRECS[prec], MODES[mode], int(factor_sweeps), int(apply_sweeps), int(restart), int(maxit),
                       float(rtol), int(max_active), 0)


_lib = None


def lib():
    """Load libabilu.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libabilu.so not built ({LIB_PATH}); run __graft_entry__.build()")
        # torch ships its own HIP runtime (soname libamdhip64.so.7). Loading torch first makes
        # libabilu bind to that same runtime instance, which owns the tensors and streams we are
        # handed; loaded first, libabilu would pull in a second runtime from the system path.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz, st = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_int
        sig = {
            "abilu_build_pattern": ([i32, vp, vp, i32, vp, C.POINTER(vp)], st),
            "abilu_pattern_destroy": ([vp], st),
            "abilu_pattern_info": ([vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i64), C.POINTER(i32),
                                    C.POINTER(i32), C.POINTER(i32)], st),
            "abilu_pattern_depth": ([vp, vp, vp, vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), vp], st),
            "abilu_factor_maxdiff": ([vp, st, vp, vp, vp, sz, C.POINTER(C.c_double), C.POINTER(C.c_double), vp], st),
            "abilu_jacobi_norms": ([vp, st, vp, vp, vp, sz, C.POINTER(C.c_double), C.POINTER(C.c_double), vp], st),
            "abilu_pattern_export": ([vp, vp, vp, vp, vp, vp], st),
            "abilu_pattern_set_chunks": ([vp, i32, i32, vp], st),
            "abilu_pattern_chunk_info": ([vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                          C.POINTER(i32), C.POINTER(i64), C.POINTER(i64)], st),
            "abilu_pattern_chunk_export": ([vp, i32, vp, vp, vp, vp], st),
            "abilu_find_lines": ([i32, vp, vp, vp, C.c_double, C.c_double, vp, vp, C.POINTER(i32)], st),
            "abilu_order": ([i32, vp, vp, vp, vp, i32, vp], st),
            "abilu_workspace_bytes": ([vp, st, i32], sz),
            "abilu_factor": ([vp, vp, vp, vp, st, i32, st, st, vp, sz, vp], st),
            "abilu_apply": ([vp, vp, vp, st, vp, vp, i32, st, vp, sz, vp], st),
            "abilu_apply_noalloc": ([vp, vp, vp, st, vp, vp, i32, st, vp], st),
            "abilu_spmv": ([vp, vp, vp, vp, vp], st),
            "abilu_factor_to_csr": ([vp, st, vp, vp, vp], st),
            "abilu_factor_from_csr": ([vp, st, vp, vp, vp], st),
            "fgmres_solve": ([vp, vp, vp, vp, i32, i32, C.c_double, vp, vp, st, i32, st, C.c_uint32, vp, sz, vp,
                              C.POINTER(FgmresResult)], st),
            "abilu_ilu_residual": ([vp, vp, vp, st, vp, sz, C.POINTER(C.c_double), vp], st),
            "abilu_read_flags": ([vp, i32, C.POINTER(C.c_uint32), vp], st),
            "abilu_clear_flags": ([vp, vp], st),
            "abilu_stream_copy": ([vp, vp, sz, vp], st),
            "abilu_profile_enable": ([i32, i32], st),
            "abilu_profile_report": ([C.c_char_p, sz], st),
            "abilu_status_string": ([st], C.c_char_p),
            "abilu_last_error": ([C.c_char_p, sz], st),
            "abilu_gen_sizes": ([C.POINTER(GenSpec), C.POINTER(i32), C.POINTER(i64)], st),
            "abilu_gen_scratch_bytes": ([C.POINTER(GenSpec)], sz),
            "abilu_gen_build": ([C.POINTER(GenSpec), vp, vp, vp, vp, vp, vp], st),
            "abilu_serve_footprint": ([C.POINTER(ServeConfig), C.POINTER(GenSpec)], sz),
            "abilu_serve_create": ([C.POINTER(ServeConfig), vp, sz, C.POINTER(vp)], st),
            "abilu_serve_destroy": ([vp], st),
            "abilu_serve_submit": ([vp, C.POINTER(Request), C.POINTER(i64)], st),
            "abilu_serve_step": ([vp, vp, C.POINTER(i32), C.POINTER(i32)], st),
            "abilu_serve_poll": ([vp, i64, C.POINTER(i32), C.POINTER(RequestResult)], st),
            "abilu_serve_run": ([vp, C.POINTER(Request), i32, C.POINTER(RequestResult), C.POINTER(C.c_double), vp],
                                st),
            "abilu_serve_stats": ([vp, C.POINTER(ServeStats)], st),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def abilu_last_error() -> str:
    buf = C.create_string_buffer(512)
    lib().abilu_last_error(buf, len(buf))
    return buf.value.decode(errors="replace")


def status_string(status: int) -> str:
    return lib().abilu_status_string(int(status)).decode()


def _check(status: int, where: str, ok=(ABILU_OK,)) -> int:
    if status not in ok:
        raise AbiluError(status, where)
    return status


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Pattern:
    """Owns an abilu_pattern handle."""

    def __init__(self, handle: int):
        self.handle = C.c_void_p(handle)

    def info(self):
        """(N, Z, npairs)."""
        n = C.c_int32(); z = C.c_int64(); npairs = C.c_int64()
        _check(lib().abilu_pattern_info(self.handle, C.byref(n), C.byref(z), C.byref(npairs), None, None, None),
               "abilu_pattern_info")
        return n.value, z.value, npairs.value

    def dependency_info(self):
        """(depth D, lower levels, upper levels) as abilu_pattern_info reports them (-1: not computed)."""
        d = C.c_int32(); ll = C.c_int32(); lu = C.c_int32()
        _check(lib().abilu_pattern_info(self.handle, None, None, None, C.byref(d), C.byref(ll), C.byref(lu)),
               "abilu_pattern_info")
        return d.value, ll.value, lu.value

    def destroy(self):
        if self.handle is not None and self.handle.value:
            lib().abilu_pattern_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def abilu_build_pattern(nbrows: int, rowptr, colidx, bs: int = 4, stream=None) -> Pattern:
    out = C.c_void_p()
    _check(lib().abilu_build_pattern(int(nbrows), _ptr(rowptr), _ptr(colidx), int(bs), _stream(stream),
                                     C.byref(out)), "abilu_build_pattern")
    return Pattern(out.value)


def abilu_pattern_export(p: Pattern, diag_pos=None, pair_ptr=None, pik=None, pkj=None, stream=None):
    _check(lib().abilu_pattern_export(p.handle, _ptr(diag_pos), _ptr(pair_ptr), _ptr(pik), _ptr(pkj),
                                      _stream(stream)), "abilu_pattern_export")


def abilu_pattern_depth(p: Pattern, depth=None, level_lower=None, level_upper=None, stream=None):
    """Dependency analysis on the device: (D, lower levels, upper levels); optional int32 device
    tensors receive the depth of every block (CSR order) and the level of every row."""
    d = C.c_int32(); ll = C.c_int32(); lu = C.c_int32()
    _check(lib().abilu_pattern_depth(p.handle, _ptr(depth), _ptr(level_lower), _ptr(level_upper), C.byref(d),
                                     C.byref(ll), C.byref(lu), _stream(stream)), "abilu_pattern_depth")
    return d.value, ll.value, lu.value


def abilu_pattern_set_chunks(p: Pattern, rows_per_chunk: int, runner: str = "auto", stream=None):
    _check(lib().abilu_pattern_set_chunks(p.handle, int(rows_per_chunk), CHUNK_RUNNERS[runner], _stream(stream)),
           "abilu_pattern_set_chunks")


def abilu_pattern_chunk_info(p: Pattern) -> dict:
    v = [C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()]
    _check(lib().abilu_pattern_chunk_info(p.handle, *[C.byref(x) for x in v]), "abilu_pattern_chunk_info")
    keys = ("rows_per_chunk", "nchunks", "runner", "max_levels_lower", "max_levels_upper", "levels_lower",
            "levels_upper")
    out = {k: x.value for k, x in zip(keys, v)}
    out["runner"] = {v: k for k, v in CHUNK_RUNNERS.items()}.get(out["runner"], None) if out["rows_per_chunk"] else None
    return out


def abilu_pattern_chunk_export(p: Pattern, upper: bool, order=None, lvptr=None, lvstart=None, stream=None):
    _check(lib().abilu_pattern_chunk_export(p.handle, int(bool(upper)), _ptr(order), _ptr(lvptr), _ptr(lvstart),
                                            _stream(stream)), "abilu_pattern_chunk_export")


ORDERINGS = {"rcm": 0, "1wd": 1, "line": 2, "line_rcm": 3, "line_1wd": 4}


def _host_i32(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.int32)


def abilu_find_lines(n: int, rowptr, colidx, weight, threshold: float = 10.0, strong_ratio: float = 4.0):
    """Lines of anisotropic cells on host arrays: (line_of int32[n], line_pos int32[n], nlines)."""
    import numpy as np
    rp, ci = _host_i32(rowptr), _host_i32(colidx)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    lo = np.empty(max(n, 1), np.int32)
    lp = np.empty(max(n, 1), np.int32)
    nl = C.c_int32()
    _check(lib().abilu_find_lines(int(n), rp.ctypes.data, ci.ctypes.data, w.ctypes.data, float(threshold),
                                  float(strong_ratio), lo.ctypes.data, lp.ctypes.data, C.byref(nl)),
           "abilu_find_lines")
    return lo[:n], lp[:n], nl.value


def abilu_order(n: int, rowptr, colidx, ordering: str, line_of=None, line_pos=None):
    """new_of_old int32[n] of an ordering computed on host arrays."""
    import numpy as np
    rp, ci = _host_i32(rowptr), _host_i32(colidx)
    lo = _host_i32(line_of) if line_of is not None else None
    lp = _host_i32(line_pos) if line_pos is not None else None
    out = np.empty(max(n, 1), np.int32)
    _check(lib().abilu_order(int(n), rp.ctypes.data, ci.ctypes.data, None if lo is None else lo.ctypes.data,
                             None if lp is None else lp.ctypes.data, ORDERINGS[ordering], out.ctypes.data),
           "abilu_order")
    return out[:n]


def abilu_workspace_bytes(p: Pattern, prec: str = "f32", fgmres_restart: int = 0) -> int:
    return int(lib().abilu_workspace_bytes(p.handle, PRECS[prec], int(fgmres_restart)))


def abilu_factor(p: Pattern, A, LU, Dinv, prec: str, nsweeps: int, mode: str, work, init: str = "A",
                 stream=None) -> int:
    return _check(lib().abilu_factor(p.handle, _ptr(A), _ptr(LU), _ptr(Dinv), PRECS[prec], int(nsweeps),
                                     MODES[mode], INITS[init], _ptr(work), work.numel() * work.element_size(),
                                     _stream(stream)), "abilu_factor")


def abilu_apply(p: Pattern, LU, Dinv, prec: str, r, z, nsweeps: int, mode: str, work, stream=None) -> int:
    return _check(lib().abilu_apply(p.handle, _ptr(LU), _ptr(Dinv), PRECS[prec], _ptr(r), _ptr(z), int(nsweeps),
                                    MODES[mode], _ptr(work), work.numel() * work.element_size(), _stream(stream)),
                  "abilu_apply")


ABILU_NOALLOC_SCRATCH_BYTES = 64 << 20


def abilu_apply_noalloc(p: Pattern, LU, Dinv, prec: str, r, z, nsweeps: int, mode: str, stream=None) -> int:
    return _check(lib().abilu_apply_noalloc(p.handle, _ptr(LU), _ptr(Dinv), PRECS[prec], _ptr(r), _ptr(z),
                                            int(nsweeps), MODES[mode], _stream(stream)), "abilu_apply_noalloc")


def abilu_factor_to_csr(p: Pattern, prec: str, LU, csr, stream=None) -> int:
    return _check(lib().abilu_factor_to_csr(p.handle, PRECS[prec], _ptr(LU), _ptr(csr), _stream(stream)),
                  "abilu_factor_to_csr")


def abilu_factor_from_csr(p: Pattern, prec: str, csr, LU, stream=None) -> int:
    return _check(lib().abilu_factor_from_csr(p.handle, PRECS[prec], _ptr(csr), _ptr(LU), _stream(stream)),
                  "abilu_factor_from_csr")


def abilu_spmv(p: Pattern, A, x, y, stream=None) -> int:
    return _check(lib().abilu_spmv(p.handle, _ptr(A), _ptr(x), _ptr(y), _stream(stream)), "abilu_spmv")


def fgmres_solve(p: Pattern, A, b, x, restart: int, maxit: int, rtol: float, LU, Dinv, prec: str,
                 apply_sweeps: int, mode: str, work, zero_guess: bool = False, stream=None):
    """Returns (status, result dict). Warnings (no convergence, modified iteration) are returned,
    errors raise."""
    res = FgmresResult()
    opts = ABILU_FGMRES_ZERO_GUESS if zero_guess else 0
    st = lib().fgmres_solve(p.handle, _ptr(A), _ptr(b), _ptr(x), int(restart), int(maxit), float(rtol), _ptr(LU),
                            _ptr(Dinv), PRECS[prec], int(apply_sweeps), MODES[mode], opts, _ptr(work),
                            work.numel() * work.element_size(), _stream(stream), C.byref(res))
    _check(st, "fgmres_solve", ok=(ABILU_OK, ABILU_WARN_MODIFIED, ABILU_WARN_NOCONV, ABILU_ENONFINITE))
    return st, res.as_dict()


def abilu_ilu_residual(p: Pattern, A, LU, prec: str, work, stream=None) -> float:
    out = C.c_double()
    _check(lib().abilu_ilu_residual(p.handle, _ptr(A), _ptr(LU), PRECS[prec], _ptr(work),
                                    work.numel() * work.element_size(), C.byref(out), _stream(stream)),
           "abilu_ilu_residual")
    return out.value


def abilu_factor_maxdiff(p: Pattern, prec: str, X, Y, work, stream=None):
    """(max |X - Y| over the strictly lower blocks, over the diagonal and upper blocks); Y double,
    both in the factor layout."""
    lo = C.c_double(); up = C.c_double()
    _check(lib().abilu_factor_maxdiff(p.handle, PRECS[prec], _ptr(X), _ptr(Y), _ptr(work),
                                      work.numel() * work.element_size(), C.byref(lo), C.byref(up), _stream(stream)),
           "abilu_factor_maxdiff")
    return lo.value, up.value


def abilu_jacobi_norms(p: Pattern, prec: str, LU, Dinv, work, stream=None):
    """(||L_strict||_inf, ||Dinv U_strict||_inf)."""
    nl = C.c_double(); nu = C.c_double()
    _check(lib().abilu_jacobi_norms(p.handle, PRECS[prec], _ptr(LU), _ptr(Dinv), _ptr(work),
                                    work.numel() * work.element_size(), C.byref(nl), C.byref(nu), _stream(stream)),
           "abilu_jacobi_norms")
    return nl.value, nu.value


def abilu_read_flags(work, clear: bool = False, stream=None) -> int:
    out = C.c_uint32()
    _check(lib().abilu_read_flags(_ptr(work), int(bool(clear)), C.byref(out), _stream(stream)), "abilu_read_flags")
    return out.value


def abilu_clear_flags(work, stream=None) -> int:
    return _check(lib().abilu_clear_flags(_ptr(work), _stream(stream)), "abilu_clear_flags")


def abilu_stream_copy(dst, src, nbytes: int, stream=None) -> int:
    return _check(lib().abilu_stream_copy(_ptr(dst), _ptr(src), int(nbytes), _stream(stream)), "abilu_stream_copy")


def abilu_profile_enable(enable: bool, max_launches: int = 65536) -> int:
    return _check(lib().abilu_profile_enable(int(bool(enable)), int(max_launches)), "abilu_profile_enable")


def abilu_profile_report() -> dict:
    buf = C.create_string_buffer(1 << 16)
    _check(lib().abilu_profile_report(buf, len(buf)), "abilu_profile_report")
    return json.loads(buf.value.decode())


def abilu_gen_sizes(req: dict):
    """(N, Z) of a generated request (host only)."""
    spec = gen_spec(req); n = C.c_int32(); z = C.c_int64()
    _check(lib().abilu_gen_sizes(C.byref(spec), C.byref(n), C.byref(z)), "abilu_gen_sizes")
    return n.value, z.value


def abilu_gen_scratch_bytes(req: dict) -> int:
    spec = gen_spec(req)
    return int(lib().abilu_gen_scratch_bytes(C.byref(spec)))


def abilu_gen_build(req: dict, rowptr, colidx, A, b, scratch, stream=None) -> int:
    spec = gen_spec(req)
    return _check(lib().abilu_gen_build(C.byref(spec), _ptr(rowptr), _ptr(colidx), _ptr(A), _ptr(b), _ptr(scratch),
                                        _stream(stream)), "abilu_gen_build")


def abilu_serve_footprint(cfg: ServeConfig, req: dict) -> int:
    """Pool bytes a request holds (host only; 0 if the config or spec is invalid)."""
    spec = gen_spec(req)
    return int(lib().abilu_serve_footprint(C.byref(cfg), C.byref(spec)))


class Server:
    """Owns an abilu_server over a caller pool (a torch uint8 tensor kept alive here)."""

    def __init__(self, cfg: ServeConfig, pool):
        self.cfg = cfg
        self.pool = pool
        out = C.c_void_p()
        _check(lib().abilu_serve_create(C.byref(cfg), _ptr(pool), pool.numel() * pool.element_size(), C.byref(out)),
               "abilu_serve_create")
        self.handle = out

    def submit(self, req: dict, x_out=None) -> int:
        r = Request(gen_spec(req), 0.0, _ptr(x_out))
        rid = C.c_int64()
        _check(lib().abilu_serve_submit(self.handle, C.byref(r), C.byref(rid)), "abilu_serve_submit")
        return rid.value

    def step(self, stream=None):
        a = C.c_int32(); q = C.c_int32()
        _check(lib().abilu_serve_step(self.handle, _stream(stream), C.byref(a), C.byref(q)), "abilu_serve_step")
        return a.value, q.value

    def poll(self, rid: int):
        done = C.c_int32(); res = RequestResult()
        _check(lib().abilu_serve_poll(self.handle, int(rid), C.byref(done), C.byref(res)), "abilu_serve_poll")
        return res.as_dict() if done.value else None

    def run(self, reqs, arrivals=None, x_outs=None, stream=None):
        """Serve a trace; returns (list of result dicts, elapsed seconds)."""
        cnt = len(reqs)
        arr = (Request * max(cnt, 1))()
        for q, rq in enumerate(reqs):
            arr[q] = Request(gen_spec(rq), float(arrivals[q]) if arrivals is not None else 0.0,
                             _ptr(x_outs[q]) if x_outs is not None else None)
        res = (RequestResult * max(cnt, 1))()
        el = C.c_double()
        _check(lib().abilu_serve_run(self.handle, arr, cnt, res, C.byref(el), _stream(stream)), "abilu_serve_run")
        return [res[q].as_dict() for q in range(cnt)], el.value

    def stats(self) -> dict:
        out = ServeStats()
        _check(lib().abilu_serve_stats(self.handle, C.byref(out)), "abilu_serve_stats")
        return out.as_dict()

    def destroy(self):
        if self.handle is not None and self.handle.value:
            lib().abilu_serve_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
