"""Dense NumPy references used to pin the oracle (independent of oracle/ and of the HIP path).

They work on the dense n x n matrix, so they are only for tiny cases.
"""
import numpy as np


def pattern_mask(n, rowptr, colidx):
    m = np.zeros((n, n), bool)
    for i in range(n):
        m[i, colidx[rowptr[i]:rowptr[i + 1]]] = True
    return m


def to_dense(n, rowptr, colidx, blocks):
    d = np.zeros((4 * n, 4 * n))
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            j = colidx[e]
            d[4 * i:4 * i + 4, 4 * j:4 * j + 4] = blocks[e]
    return d


def factors_dense(n, rowptr, colidx, X):
    """Dense unit block-lower L and block-upper U from the combined factor array."""
    L = np.eye(4 * n)
    U = np.zeros((4 * n, 4 * n))
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            j = colidx[e]
            if j < i:
                L[4 * i:4 * i + 4, 4 * j:4 * j + 4] = X[e]
            else:
                U[4 * i:4 * i + 4, 4 * j:4 * j + 4] = X[e]
    return L, U


def block_ilu0_kij(n, rowptr, colidx, A):
    """Static-pattern block ILU(0) by right-looking (KIJ) Gaussian elimination with dropping:
    for k: for i > k in pattern: A_ik <- A_ik A_kk^{-1}; for j > k with (k,j) and (i,j) in the
    pattern: A_ij <- A_ij - A_ik A_kj. Returns the factor blocks in CSR order."""
    mask = pattern_mask(n, rowptr, colidx)
    blk = {}
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            blk[(i, int(colidx[e]))] = A[e].copy()
    for k in range(n):
        inv_kk = np.linalg.inv(blk[(k, k)])
        for i in range(k + 1, n):
            if not mask[i, k]:
                continue
            blk[(i, k)] = blk[(i, k)] @ inv_kk
            for j in range(k + 1, n):
                if mask[k, j] and mask[i, j]:
                    blk[(i, j)] = blk[(i, j)] - blk[(i, k)] @ blk[(k, j)]
    out = np.empty_like(A)
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            out[e] = blk[(i, int(colidx[e]))]
    return out


def rel(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    d = np.linalg.norm((a - b).ravel())
    s = np.linalg.norm(b.ravel())
    return d / s if s > 0 else d


def block_rel(a, b):
    """Relative error of every block: ||a_k - b_k||_F / ||b_k||_F over the leading axis (a block
    of b with zero norm gives its absolute error)."""
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    a = a.reshape(len(b), -1); b = b.reshape(len(b), -1)
    dn = np.linalg.norm(a - b, axis=1)
    bn = np.linalg.norm(b, axis=1)
    return np.where(bn > 0, dn / np.where(bn > 0, bn, 1.0), dn)


def assert_same_bits(a, b, what=""):
    """Bit-for-bit equality (signed zeros compare equal), with the size of any difference."""
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if not np.array_equal(a, b):
        bad = a != b
        raise AssertionError(f"{what}: {int(bad.sum())} of {a.size} values differ; relative error {rel(a, b):.3e}, "
                             f"largest absolute difference {np.abs(a - b)[bad].max():.3e}")
