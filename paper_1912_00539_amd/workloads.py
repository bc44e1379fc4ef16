"""Seeded synthetic 4x4-block sparse (BSR) Jacobians shaped like the paper's test cases.

This module only generates inputs. It holds none of the preconditioner's arithmetic and is the
one piece of code shared by the HIP path's tests/benchmarks and the CPU oracle's tests.

What the paper fixes about the matrices (Section 2, "The solver setup"):
  * cell-centred finite volumes on 2-D grids; the d+2 = 4 conserved variables of a cell are
    numbered consecutively, so the Jacobian is made of dense 4x4 blocks, one block row per cell
    and one off-diagonal block per face neighbour;
  * the pseudo-time term adds V_i / dtau_i * I to each diagonal block, with
    dtau_i = CFL * V_i / sum_f nu_f a_f (local time step equation), so the shift is
    sum_f nu_f a_f / CFL and the cell volume cancels;
  * the blocks of one block are stored contiguously (we use row-major 4x4).
The paper's meshes, flow states and Jacobians are not available, so the block values are drawn
from a counter-based generator:
  * each face f gets one weight w_f ~ U(0.5, 1.5) shared by A_ij and A_ji;
  * the 16 entries of A_ij and of A_ji are drawn independently from U(-1, 1) and scaled by w_f
    (a nonsymmetric Jacobian on a structurally symmetric pattern);
  * the diagonal block is (s_i + sum_j ||A_ij||_1) I + P_i, with P_i ~ U(-0.1, 0.1)^{4x4} and
    ||.||_1 the induced 1-norm (max absolute column sum). s_i is either a constant, or the
    pseudo-time shift sum_j ||A_ij||_1 / CFL, with ||A_ij||_1 standing in for nu_f a_f;
  * the right-hand side is U(-1, 1).
Orderings (Section 5): natural lexicographic, random permutation followed by reverse
Cuthill-McKee (RCM), and line ordering (the cells of each wall-normal line contiguous, walking
from the wall outward).

Random numbers come from a counter-based hash: value = mix(key(seed, stream) + GOLDEN * index),
the SplitMix64 finaliser (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014). Every random number is keyed by the *natural* (pre-ordering) face or cell id, so a
re-ordered case holds exactly the same matrix, only permuted.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# random streams
S_FACE_W, S_OFFDIAG, S_DIAGPERT, S_RHS, S_SPLIT, S_PERM, S_DRIFT = 1, 2, 3, 4, 5, 6, 7

BS = 4  # block size b = d + 2 for d = 2


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k = np.array([(int(seed) * 0x9E3779B97F4A7C15 + int(stream) * 0xD1B54A32D192ED03) & (2**64 - 1)],
                     dtype=np.uint64)
        return _mix64(k)[0]


def uniform01(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """U[0,1) doubles for counters idx (uint64-convertible), 53-bit resolution."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _key(seed, stream) + idx * GOLDEN
        h = _mix64(z)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform(seed: int, stream: int, idx: np.ndarray, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, stream, idx)


# --------------------------------------------------------------------------- meshes
@dataclasses.dataclass
class Mesh:
    """Face-adjacency graph of a 2-D cell mesh, in natural numbering."""
    ncells: int
    fa: np.ndarray          # int64 [F] first cell of face
    fb: np.ndarray          # int64 [F] second cell of face (fa < fb not required)
    fscale: np.ndarray      # float64 [F] extra face-weight factor (anisotropy), 1 if isotropic
    kind: str
    shape: tuple


def quad_mesh(nx: int, ny: int) -> Mesh:
    """nx x ny structured quads, 5-point face stencil, cell id = iy*nx + ix."""
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    cid = (iy * nx + ix).astype(np.int64)
    h_a = cid[:, :-1].ravel(); h_b = cid[:, 1:].ravel()
    v_a = cid[:-1, :].ravel(); v_b = cid[1:, :].ravel()
    fa = np.concatenate([h_a, v_a]); fb = np.concatenate([h_b, v_b])
    return Mesh(nx * ny, fa, fb, np.ones(fa.size), "quad", (nx, ny))


def aniso_quad_mesh(n_tan: int, n_norm: int, ar_wall: float = 1000.0) -> Mesh:
    """Boundary-layer-like quads: n_tan cells along the wall, n_norm wall-normal layers.

    Layer k (0 at the wall) has aspect ratio AR_k = ar_wall^(1 - k/(n_norm-1)). A wall-normal face
    between layers k and k+1 is scaled by sqrt(AR_k AR_{k+1}); tangential faces are unscaled.
    Natural cell id = k * n_tan + t (wall-tangential index fastest).
    """
    t, k = np.meshgrid(np.arange(n_tan), np.arange(n_norm), indexing="xy")
    cid = (k * n_tan + t).astype(np.int64)
    if n_norm > 1:
        ar = ar_wall ** (1.0 - np.arange(n_norm) / (n_norm - 1))
    else:
        ar = np.array([ar_wall])
    h_a = cid[:, :-1].ravel(); h_b = cid[:, 1:].ravel()
    v_a = cid[:-1, :].ravel(); v_b = cid[1:, :].ravel()
    v_scale = np.sqrt(ar[:-1] * ar[1:])[:, None].repeat(n_tan, axis=1).ravel()
    fa = np.concatenate([h_a, v_a]); fb = np.concatenate([h_b, v_b])
    fs = np.concatenate([np.ones(h_a.size), v_scale])
    return Mesh(n_tan * n_norm, fa, fb, fs, "aniso_quad", (n_tan, n_norm))


def split_tri_mesh(nx: int, ny: int, seed: int) -> Mesh:
    """nx x ny quads, each cut into two triangles along a seeded random diagonal.

    Quad q = iy*nx + ix holds triangles 2q and 2q+1. With diagonal '/' (0,0)-(1,1) triangle 2q is
    the lower-right one (bottom, right edges) and 2q+1 the upper-left (top, left); with '\\'
    (1,0)-(0,1) triangle 2q is lower-left (bottom, left) and 2q+1 upper-right (top, right).
    Each triangle has at most 3 face neighbours. Vertex jitter does not enter the matrix.
    """
    nq = nx * ny
    q = np.arange(nq, dtype=np.int64)
    diag = uniform01(seed, S_SPLIT, q) < 0.5          # True: '\' diagonal
    t0 = 2 * q; t1 = 2 * q + 1
    bottom = t0; top = t1
    left = np.where(diag, t0, t1); right = np.where(diag, t1, t0)
    qid = q.reshape(ny, nx)
    # internal diagonal faces
    fa = [t0]; fb = [t1]
    # horizontal neighbours: right edge of (ix,iy) with left edge of (ix+1,iy)
    a = qid[:, :-1].ravel(); b = qid[:, 1:].ravel()
    fa.append(right[a]); fb.append(left[b])
    # vertical neighbours: top of (ix,iy) with bottom of (ix,iy+1)
    a = qid[:-1, :].ravel(); b = qid[1:, :].ravel()
    fa.append(top[a]); fb.append(bottom[b])
    fa = np.concatenate(fa); fb = np.concatenate(fb)
    return Mesh(2 * nq, fa, fb, np.ones(fa.size), "tri", (nx, ny))


def nine_point_mesh(nx: int, ny: int) -> Mesh:
    """Structured grid with 8 neighbours per cell (edge + corner); has triangles in its graph,
    so the block ILU(0) update sets K(i,j) are non-empty off the diagonal."""
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    cid = (iy * nx + ix).astype(np.int64)
    fa, fb = [], []
    for dx, dy in ((1, 0), (0, 1), (1, 1), (1, -1)):
        x0, x1 = max(0, -dx), nx - max(0, dx)
        y0, y1 = max(0, -dy), ny - max(0, dy)
        a = cid[y0:y1, x0:x1].ravel()
        b = cid[y0 + dy:y1 + dy, x0 + dx:x1 + dx].ravel()
        fa.append(a); fb.append(b)
    fa = np.concatenate(fa); fb = np.concatenate(fb)
    return Mesh(nx * ny, fa, fb, np.ones(fa.size), "nine_point", (nx, ny))


def random_graph_mesh(ncells: int, avg_deg: float, seed: int) -> Mesh:
    """Random symmetric pattern (Erdos-Renyi-like face graph), for generic pattern coverage."""
    npairs = ncells * (ncells - 1) // 2
    m = min(npairs, int(round(avg_deg * ncells / 2)))
    if m == 0 or ncells < 2:
        z = np.zeros(0, np.int64)
        return Mesh(ncells, z, z, np.zeros(0), "random", (ncells,))
    u = uniform01(seed, S_PERM, np.arange(4 * m + 16))
    a = (u[0::2][: 2 * m + 8] * ncells).astype(np.int64)
    b = (u[1::2][: 2 * m + 8] * ncells).astype(np.int64)
    keep = a != b
    a, b = np.minimum(a[keep], b[keep]), np.maximum(a[keep], b[keep])
    key = np.unique(a * ncells + b)[:m]
    return Mesh(ncells, key // ncells, key % ncells, np.ones(key.size), "random", (ncells,))


def chain_mesh(ncells: int) -> Mesh:
    """1-D line of cells: block tridiagonal, ILU(0) has no dropped fill (it is exact LU)."""
    a = np.arange(ncells - 1, dtype=np.int64)
    return Mesh(ncells, a, a + 1, np.ones(a.size), "chain", (ncells,))


# --------------------------------------------------------------------------- orderings
def rcm_order(mesh: Mesh, seed: int, permute_first: bool = True) -> np.ndarray:
    """new_of_old permutation: optional seeded random permutation, then reverse Cuthill-McKee."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    n = mesh.ncells
    if permute_first:
        perm = np.argsort(uniform01(seed, S_PERM, np.arange(n)), kind="stable")  # position -> old
        inv = np.empty(n, np.int64); inv[perm] = np.arange(n)                     # old -> position
    else:
        inv = np.arange(n, dtype=np.int64)
    a = inv[mesh.fa]; b = inv[mesh.fb]
    g = sp.coo_matrix((np.ones(2 * a.size, np.int8), (np.concatenate([a, b]), np.concatenate([b, a]))),
                      shape=(n, n)).tocsr()
    rcm = np.asarray(reverse_cuthill_mckee(g, symmetric_mode=True), dtype=np.int64)  # new -> position
    pos_to_new = np.empty(n, np.int64); pos_to_new[rcm] = np.arange(n)
    return pos_to_new[inv]


def line_order(mesh: Mesh) -> np.ndarray:
    """Wall-normal lines contiguous: for the anisotropic quad mesh, new id = t*n_norm + k."""
    assert mesh.kind == "aniso_quad"
    n_tan, n_norm = mesh.shape
    old = np.arange(mesh.ncells, dtype=np.int64)
    k = old // n_tan; t = old % n_tan
    return t * n_norm + k


def natural_order(mesh: Mesh) -> np.ndarray:
    return np.arange(mesh.ncells, dtype=np.int64)


# --------------------------------------------------------------------------- BSR assembly
@dataclasses.dataclass
class BSRCase:
    """A = BSR matrix with 4x4 row-major blocks; b = right-hand side (length 4N)."""
    n: int                   # block rows (cells)
    rowptr: np.ndarray       # int32 [N+1]
    colidx: np.ndarray       # int32 [Z], ascending within each row, diagonal present
    vals: np.ndarray         # float64 [Z, 4, 4]
    b: np.ndarray            # float64 [4N]
    meta: dict

    @property
    def nnzb(self) -> int:
        return int(self.colidx.size)

    def dense(self) -> np.ndarray:
        d = np.zeros((4 * self.n, 4 * self.n))
        for i in range(self.n):
            for e in range(self.rowptr[i], self.rowptr[i + 1]):
                j = self.colidx[e]
                d[4 * i:4 * i + 4, 4 * j:4 * j + 4] = self.vals[e]
        return d


def _block_1norm(blocks: np.ndarray) -> np.ndarray:
    return np.abs(blocks).sum(axis=1).max(axis=1)     # max over columns of abs column sums


def assemble(mesh: Mesh, new_of_old: np.ndarray, seed: int, shift: str = "const", s: float = 1.0,
             cfl: float = 100.0, chunk: int = 1 << 21) -> BSRCase:
    """Build the BSR Jacobian for `mesh` in the ordering `new_of_old`.

    shift='const': s_i = s.  shift='cfl': s_i = sum_j ||A_ij||_1 / cfl.
    """
    n = mesh.ncells
    F = mesh.fa.size
    nz = n + 2 * F
    # directed couplings: face f gives (fa -> fb) with counter 2f and (fb -> fa) with counter 2f+1
    rows_old = np.concatenate([mesh.fa, mesh.fb])
    cols_old = np.concatenate([mesh.fb, mesh.fa])
    ctr = np.concatenate([2 * np.arange(F, dtype=np.int64), 2 * np.arange(F, dtype=np.int64) + 1])
    w = uniform(seed, S_FACE_W, np.arange(F, dtype=np.int64), 0.5, 1.5) * mesh.fscale
    wdir = np.concatenate([w, w])
    off = np.empty((2 * F, BS, BS), np.float64)
    ent = np.arange(16, dtype=np.uint64)
    for c0 in range(0, 2 * F, chunk):
        c1 = min(2 * F, c0 + chunk)
        idx = (ctr[c0:c1].astype(np.uint64)[:, None] * np.uint64(16) + ent[None, :])
        off[c0:c1] = (uniform(seed, S_OFFDIAG, idx, -1.0, 1.0) * wdir[c0:c1, None]).reshape(-1, BS, BS)
    # diagonal
    nrm = np.zeros(n)
    if F:
        nrm += np.bincount(rows_old, weights=_block_1norm(off), minlength=n)
    if shift == "const":
        sh = np.full(n, float(s))
    elif shift == "cfl":
        sh = nrm / float(cfl)
    else:
        raise ValueError(shift)
    diag = np.empty((n, BS, BS))
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        idx = np.arange(c0, c1, dtype=np.uint64)[:, None] * np.uint64(16) + ent[None, :]
        diag[c0:c1] = uniform(seed, S_DIAGPERT, idx, -0.1, 0.1).reshape(-1, BS, BS)
    diag += (sh + nrm)[:, None, None] * np.eye(BS)[None]
    rhs_old = uniform(seed, S_RHS, np.arange(4 * n, dtype=np.int64), -1.0, 1.0).reshape(n, BS)
    # permute and sort into CSR order
    new = np.asarray(new_of_old, dtype=np.int64)
    r = np.concatenate([new[np.arange(n)], new[rows_old]])
    c = np.concatenate([new[np.arange(n)], new[cols_old]])
    key = r * n + c
    order = np.argsort(key, kind="stable")
    colidx = c[order].astype(np.int32)
    counts = np.bincount(r, minlength=n)
    rowptr = np.zeros(n + 1, np.int64); np.cumsum(counts, out=rowptr[1:])
    vals = np.empty((nz, BS, BS))
    is_diag = order < n
    vals[is_diag] = diag[order[is_diag]]
    vals[~is_diag] = off[order[~is_diag] - n]
    b = np.empty((n, BS)); b[new] = rhs_old
    return BSRCase(n, rowptr.astype(np.int32), colidx, vals, b.ravel(),
                   dict(kind=mesh.kind, shape=mesh.shape, seed=seed, shift=shift, s=s, cfl=cfl))


def block_face_weights(mesh: Mesh, new_of_old: np.ndarray, rowptr: np.ndarray, colidx: np.ndarray) -> np.ndarray:
    """Geometric coupling of each block of a case assembled from `mesh` in the ordering
    `new_of_old`: the face's anisotropy scale (1 for an isotropic face, sqrt(AR_k AR_{k+1}) for a
    wall-normal face of the boundary-layer mesh), 0 on the diagonal. This is the cell-geometry
    input of line finding (face area over centroid distance, up to a constant)."""
    new = np.asarray(new_of_old, np.int64)
    n = mesh.ncells
    a = new[mesh.fa]; b = new[mesh.fb]
    r = np.concatenate([a, b]); c = np.concatenate([b, a])
    w = np.concatenate([mesh.fscale, mesh.fscale])
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    key_blk = rows * n + np.asarray(colidx, np.int64)
    pos = np.searchsorted(key_blk, r * n + c)
    out = np.zeros(colidx.size)
    out[pos] = w
    return out


# --------------------------------------------------------------------------- named cases
def case(name: str, seed: int = 0, **kw) -> BSRCase:
    """Named workloads.

    'quad32'      32x32 quads, 5-point, natural order, s = 1           (1,024 cells)
    'tri300'      300x300 split quads -> 180,000 triangles, permuted + RCM, CFL shift
    'aniso1000'   1000 x 500 anisotropic quads (AR 1000 at the wall), line order or RCM
    'tri2000'     2000x1000 split quads -> 4,000,000 triangles, permuted + RCM, CFL 100
    Small variants for parity tests: 'quad', 'tri', 'aniso', 'nine', 'random', 'chain' with
    explicit sizes in kw.
    """
    if name == "quad32":
        return assemble(quad_mesh(32, 32), natural_order(quad_mesh(32, 32)), seed, "const", s=1.0)
    if name == "tri300":
        cfl = kw.get("cfl", 100.0)
        m = split_tri_mesh(300, 300, seed)
        return assemble(m, rcm_order(m, seed), seed, "cfl", cfl=cfl)
    if name == "aniso1000":
        m = aniso_quad_mesh(1000, 500)
        order = line_order(m) if kw.get("order", "line") == "line" else rcm_order(m, seed)
        return assemble(m, order, seed, "cfl", cfl=kw.get("cfl", 100.0))
    if name == "tri2000":
        m = split_tri_mesh(2000, 1000, seed)
        return assemble(m, rcm_order(m, seed), seed, "cfl", cfl=kw.get("cfl", 100.0))
    # parametrised small cases
    order = kw.get("order", "natural")
    if name == "quad":
        m = quad_mesh(kw["nx"], kw["ny"])
    elif name == "tri":
        m = split_tri_mesh(kw["nx"], kw["ny"], seed)
    elif name == "aniso":
        m = aniso_quad_mesh(kw["nx"], kw["ny"], kw.get("ar", 1000.0))
    elif name == "nine":
        m = nine_point_mesh(kw["nx"], kw["ny"])
    elif name == "random":
        m = random_graph_mesh(kw["n"], kw.get("deg", 4.0), seed)
    elif name == "chain":
        m = chain_mesh(kw["n"])
    else:
        raise KeyError(name)
    if order == "natural":
        o = natural_order(m)
    elif order == "rcm":
        o = rcm_order(m, seed)
    elif order == "line":
        o = line_order(m)
    elif order == "random":
        o = np.argsort(np.argsort(uniform01(seed, S_PERM, np.arange(m.ncells)), kind="stable"), kind="stable")
    else:
        raise KeyError(order)
    sh = kw.get("shift", "const")
    return assemble(m, o, seed, sh, s=kw.get("s", 1.0), cfl=kw.get("cfl", 100.0))


def serving_requests(count: int, seed: int):
    """Request mix for the serving workload: mesh kind 50/50 (split-quad triangles or anisotropic
    quads), cell count log-uniform in [1e4, 1e6], CFL ~ U(10, 1000); one seed per request."""
    i = np.arange(count, dtype=np.int64)
    kind = np.where(uniform01(seed, 11, i) < 0.5, "tri", "aniso")
    cells = np.exp(np.log(1e4) + (np.log(1e6) - np.log(1e4)) * uniform01(seed, 12, i))
    cfl = uniform(seed, 13, i, 10.0, 1000.0)
    out = []
    for q in range(count):
        c = float(cells[q])
        if kind[q] == "tri":
            ny = max(2, int(round(math.sqrt(c / 4.0)))); nx = max(2, int(round(c / (2.0 * ny))))
        else:
            ny = max(2, int(round(math.sqrt(c / 2.0)))); nx = max(2, int(round(c / ny)))
        out.append(dict(kind=str(kind[q]), nx=nx, ny=ny, cfl=float(cfl[q]), seed=int(seed * 100003 + q)))
    return out


def request_case(req: dict, order: str = "device") -> BSRCase:
    """Host twin of a serving request. order='device' uses the device generator's numbering
    (natural for triangles, line order for anisotropic quads); 'rcm' reorders triangles by RCM."""
    if req["kind"] == "tri":
        m = split_tri_mesh(req["nx"], req["ny"], req["seed"])
        o = rcm_order(m, req["seed"]) if order == "rcm" else natural_order(m)
        return assemble(m, o, req["seed"], "cfl", cfl=req["cfl"])
    m = aniso_quad_mesh(req["nx"], req["ny"])
    return assemble(m, line_order(m), req["seed"], "cfl", cfl=req["cfl"])


# --------------------------------------------------------------------------- pseudo-time sequences
def cfl_ramp(steps: int, cfl0: float = 10.0, growth: float = 1.5, cfl_max: float = 1000.0) -> np.ndarray:
    """CFL_t = min(cfl0 * growth^t, cfl_max): the geometric ramp of a pseudo-transient continuation
    (Section 2, local time stepping with a growing CFL number)."""
    return np.minimum(cfl0 * growth ** np.arange(steps, dtype=np.float64), cfl_max)


def jacobian_sequence(case: BSRCase, cfls, drift: float = 0.01, seed: int = 0):
    """Jacobians of successive pseudo-time steps on `case`'s pattern (yields (vals, b) per step).

    Step 0 is `case` with its diagonal shift recomputed for cfls[0]. Each later step multiplies
    every off-diagonal entry by (1 + drift u), u ~ U(-1,1) drawn per (step, entry) (a slowly
    changing flow state), and recomputes the diagonal blocks for the new neighbours and CFL:
    A_ii(t) = A_ii(0) + (c_i(t) - c_i(0)) I with c_i = sum_j ||A_ij||_1 (1 + 1/CFL). The right-hand
    side is b(0) (1 + drift u) per step. Values only; the pattern never changes.
    """
    n, z = case.n, case.nnzb
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(case.rowptr.astype(np.int64)))
    diag = case.colidx.astype(np.int64) == rows
    off = ~diag
    vals = case.vals.copy()

    def row_norms(v):
        return np.bincount(rows[off], weights=_block_1norm(v[off]), minlength=n)

    nrm0 = row_norms(vals)
    cfl0 = float(case.meta.get("cfl", 100.0)) if case.meta.get("shift") == "cfl" else None
    # c_i of the case as generated (constant shift s when the case was not CFL-shifted)
    c0 = nrm0 * (1.0 + 1.0 / cfl0) if cfl0 else nrm0 + float(case.meta.get("s", 1.0))
    eye = np.eye(4)
    ent = np.arange(16, dtype=np.uint64)
    for t, cfl in enumerate(cfls):
        if t > 0:
            idx = (np.uint64(t) * np.uint64(z) + np.arange(z, dtype=np.uint64))[:, None] * np.uint64(16) + ent[None, :]
            u = uniform(seed, S_DRIFT, idx.ravel(), -1.0, 1.0).reshape(z, 4, 4)
            vals[off] *= 1.0 + drift * u[off]
        ct = row_norms(vals) * (1.0 + 1.0 / float(cfl))
        vt = vals.copy()
        vt[diag] = case.vals[diag] + (ct - c0)[:, None, None] * eye[None]
        rb = uniform(seed, S_DRIFT, (np.uint64(t) << np.uint64(40)) + np.arange(4 * n, dtype=np.uint64), -1.0, 1.0)
        yield vt, case.b * (1.0 + drift * rb)
