"""Device-resident system: uploads a BSR case, builds the pattern and owns the factor, workspace
and vectors as torch tensors (plumbing only; every operation calls libabilu)."""
from __future__ import annotations

import numpy as np

from . import abilu as L


class DeviceSystem:
    def __init__(self, case, prec: str = "f32", restart: int = 30, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.case = case
        self.prec = prec
        self.restart = restart
        dev = torch.device(device)
        self.device = dev
        self.n = int(case.n)
        self.nnzb = int(case.nnzb)
        self.rowptr = torch.from_numpy(np.ascontiguousarray(case.rowptr, np.int32)).to(dev)
        self.colidx = torch.from_numpy(np.ascontiguousarray(case.colidx, np.int32)).to(dev)
        self.A = torch.from_numpy(np.ascontiguousarray(case.vals, np.float64).reshape(-1)).to(dev)
        self.b = torch.from_numpy(np.ascontiguousarray(case.b, np.float64)).to(dev)
        self.pattern = L.abilu_build_pattern(self.n, self.rowptr, self.colidx)
        dt = torch.float32 if prec == "f32" else torch.float64
        self.LU = torch.zeros(max(self.nnzb, 1) * 16, dtype=dt, device=dev)
        self.Dinv = torch.zeros(max(self.n, 1) * 16, dtype=dt, device=dev)
        nbytes = L.abilu_workspace_bytes(self.pattern, prec, restart)
        self.work = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self.x = torch.zeros(max(4 * self.n, 1), dtype=torch.float64, device=dev)

    def set_chunks(self, rows_per_chunk: int, runner: str = "auto"):
        """Build the chunk schedule of the chunked modes ("chunk_sync", "chunk_async")."""
        L.abilu_pattern_set_chunks(self.pattern, rows_per_chunk, runner)
        return L.abilu_pattern_chunk_info(self.pattern)

    def load_values(self, vals, b=None):
        """Replace A (and b) by new values on the same pattern (the next Jacobian of a sequence)."""
        t = self.torch
        self.A.copy_(t.from_numpy(np.ascontiguousarray(vals, np.float64).reshape(-1)))
        if b is not None:
            self.b.copy_(t.from_numpy(np.ascontiguousarray(b, np.float64)))

    def factor(self, nsweeps: int, mode: str = "sync", init: str = "A", stream=None):
        return L.abilu_factor(self.pattern, self.A, self.LU, self.Dinv, self.prec, nsweeps, mode, self.work,
                              init=init, stream=stream)

    def apply(self, r, z, nsweeps: int, mode: str = "sync", stream=None):
        return L.abilu_apply(self.pattern, self.LU, self.Dinv, self.prec, r, z, nsweeps, mode, self.work,
                             stream=stream)

    def spmv(self, x, y, stream=None):
        return L.abilu_spmv(self.pattern, self.A, x, y, stream=stream)

    def solve(self, apply_sweeps: int = 3, mode: str = "sync", rtol: float = 1e-2, maxit: int = 2500,
              x0=None, restart: int = None, stream=None):
        """FGMRES from x0 (None: zero initial guess, no initial SpMV)."""
        if x0 is not None:
            self.x.copy_(x0)
        return L.fgmres_solve(self.pattern, self.A, self.b, self.x, restart or self.restart, maxit, rtol, self.LU,
                              self.Dinv, self.prec, apply_sweeps, mode, self.work, zero_guess=x0 is None,
                              stream=stream)

    def ilu_residual(self, stream=None) -> float:
        return L.abilu_ilu_residual(self.pattern, self.A, self.LU, self.prec, self.work, stream=stream)

    def flags(self, clear: bool = False) -> int:
        return L.abilu_read_flags(self.work, clear)

    def factor_host(self):
        """(X [Z,4,4] in CSR block order, Dinv [N,4,4]) as float64 numpy arrays."""
        csr = self.torch.empty_like(self.LU)
        L.abilu_factor_to_csr(self.pattern, self.prec, self.LU, csr)
        X = csr[: self.nnzb * 16].double().cpu().numpy().reshape(self.nnzb, 4, 4)
        D = self.Dinv[: self.n * 16].double().cpu().numpy().reshape(self.n, 4, 4)
        return X, D

    def set_factor(self, X, D):
        """Load a factor given in CSR block order (rounded to the factor precision)."""
        t = self.torch
        csr = t.from_numpy(np.ascontiguousarray(X, np.float64).reshape(-1)).to(self.device).to(self.LU.dtype)
        L.abilu_factor_from_csr(self.pattern, self.prec, csr, self.LU)
        self.Dinv[: self.n * 16].copy_(t.from_numpy(np.ascontiguousarray(D, np.float64).reshape(-1)))
