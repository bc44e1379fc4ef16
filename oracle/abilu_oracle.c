/*
 * CPU FP64 oracle for the asynchronous block ILU(0) preconditioner (Kashi & Nadarajah,
 * "An asynchronous incomplete block LU preconditioner for computational fluid dynamics on
 * unstructured grids", arXiv:1912.00539).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or load this file:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use it. It shares no
 * code, header, table or helper with the HIP library.
 *
 * Plain, slow, obviously correct: every loop follows the paper's definitions directly, in
 * double precision, with no blocking or fusion. Matrices are block-sparse (BSR) with b = 4:
 * rowptr[N+1], colidx[Z] (ascending per row, diagonal present), values [Z][4][4] row-major.
 * The combined factor array X has A's pattern: X_ij = L_ij for i > j (L has an implicit identity
 * block diagonal), X_ij = U_ij for i <= j. Dinv[N][4][4] holds U_jj^{-1}.
 *
 * Readings of points the paper leaves open (each is listed with the design notes):
 *  - the initial factor guess is A itself, for L too (Section 3.3 and Section 6 setup);
 *  - a synchronous sweep uses the previous iterate's diagonal inverses (Jacobi-type iteration,
 *    equation for x^{p+1} = h(x^p) in Section 4.2);
 *  - the "arbitrary nonsingular matrix" of the modified iteration (Section 4.2, Theorem 8) is the
 *    identity, used when Gaussian elimination meets an exactly zero pivot or the inverse is not
 *    finite; flag bit 1 is then raised;
 *  - "n apply sweeps" means n forward and n backward sweeps, each from a zero initial guess.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BS 4
#define BB 16

#define ORACLE_FLAG_MODIFIED 1u
#define ORACLE_FLAG_NONFINITE 2u

/* ------------------------------------------------------------------ small dense helpers */

/* position of block (i,j) in row i, or -1 (linear scan: plain and obviously correct) */
static long find_block(const int *rowptr, const int *colidx, int i, int j) {
    for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
        if (colidx[e] == j) return e;
    return -1;
}

/* C = X * Y for 4x4 row-major blocks */
static void mat_mul(double *C, const double *X, const double *Y) {
    for (int r = 0; r < BS; ++r)
        for (int c = 0; c < BS; ++c) {
            double s = 0.0;
            for (int m = 0; m < BS; ++m) s += X[r * BS + m] * Y[m * BS + c];
            C[r * BS + c] = s;
        }
}

/* T = T - X * Y */
static void mat_sub_mul(double *T, const double *X, const double *Y) {
    double P[BB];
    mat_mul(P, X, Y);
    for (int q = 0; q < BB; ++q) T[q] -= P[q];
}

static void mat_identity(double *M) {
    for (int q = 0; q < BB; ++q) M[q] = (q % (BS + 1) == 0) ? 1.0 : 0.0;
}

/*
 * Inverse of a 4x4 block by Gaussian elimination with partial pivoting on the augmented system
 * [M | I], followed by back substitution (the exact small-block inversion of Section 4.1).
 * Returns 0 on success. If a pivot is exactly zero or the result is not finite, writes the
 * identity (the modified iteration of Section 4.2) and returns ORACLE_FLAG_MODIFIED.
 */
int oracle_inv4(const double *Min, double *Inv) {
    double M[BS][BS], R[BS][BS];
    for (int r = 0; r < BS; ++r)
        for (int c = 0; c < BS; ++c) {
            M[r][c] = Min[r * BS + c];
            R[r][c] = (r == c) ? 1.0 : 0.0;
        }
    for (int k = 0; k < BS; ++k) {
        int p = k;
        double best = fabs(M[k][k]);
        for (int r = k + 1; r < BS; ++r)
            if (fabs(M[r][k]) > best) { best = fabs(M[r][k]); p = r; }
        if (p != k)
            for (int c = 0; c < BS; ++c) {
                double t = M[k][c]; M[k][c] = M[p][c]; M[p][c] = t;
                t = R[k][c]; R[k][c] = R[p][c]; R[p][c] = t;
            }
        if (M[k][k] == 0.0) { mat_identity(Inv); return ORACLE_FLAG_MODIFIED; }
        for (int r = k + 1; r < BS; ++r) {
            double f = M[r][k] / M[k][k];
            for (int c = 0; c < BS; ++c) {
                M[r][c] -= f * M[k][c];
                R[r][c] -= f * R[k][c];
            }
        }
    }
    for (int k = BS - 1; k >= 0; --k)
        for (int c = 0; c < BS; ++c) {
            double s = R[k][c];
            for (int m = k + 1; m < BS; ++m) s -= M[k][m] * R[m][c];
            R[k][c] = s / M[k][k];
        }
    for (int r = 0; r < BS; ++r)
        for (int c = 0; c < BS; ++c)
            if (!isfinite(R[r][c])) { mat_identity(Inv); return ORACLE_FLAG_MODIFIED; }
    for (int r = 0; r < BS; ++r)
        for (int c = 0; c < BS; ++c) Inv[r * BS + c] = R[r][c];
    return 0;
}

/* ------------------------------------------------------------------ pattern analysis */

/* 0 if the pattern is valid BSR for ILU(0): rowptr monotone from 0, columns in range and
 * strictly ascending per row, every diagonal block present. -2 otherwise. */
int oracle_check_pattern(int n, const int *rowptr, const int *colidx) {
    if (n < 0) return -1;
    if (rowptr[0] != 0) return -2;
    for (int i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return -2;
        int has_diag = 0;
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (colidx[e] < 0 || colidx[e] >= n) return -2;
            if (e > rowptr[i] && colidx[e] <= colidx[e - 1]) return -2;
            if (colidx[e] == i) has_diag = 1;
        }
        if (!has_diag) return -2;
    }
    return 0;
}

/*
 * Update sets of the block ILU(0) equations (Section 4.2, block form of the Chow-Patel
 * equations): for block (i,j) in S_B, K(i,j) = { k < min(i,j) : (i,k) in S_B and (k,j) in S_B }.
 * pair_ptr[Z+1] is the CSR offset of each block's list; pik/pkj hold the positions of (i,k)
 * and (k,j), ascending in k. Call with pik == NULL to only count.
 */
long oracle_pairs(int n, const int *rowptr, const int *colidx, long *pair_ptr, int *pik, int *pkj) {
    long cnt = 0;
    for (int i = 0; i < n; ++i)
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int j = colidx[e];
            int lim = i < j ? i : j;
            pair_ptr[e] = cnt;
            for (long f = rowptr[i]; f < rowptr[i + 1]; ++f) {
                int k = colidx[f];
                if (k >= lim) continue;
                long g = find_block(rowptr, colidx, k, j);
                if (g < 0) continue;
                if (pik) { pik[cnt] = (int)f; pkj[cnt] = (int)g; }
                ++cnt;
            }
        }
    pair_ptr[rowptr[n]] = cnt;
    return cnt;
}

/*
 * Dependency depth of every block unknown (Lemma 2: in the block Gaussian-elimination ordering
 * h is strictly lower triangular, so depths are well defined). H_ij reads X_ik, X_kj for
 * k in K(i,j), and X_jj when i > j. depth = 1 + max depth of what it reads (1 if nothing).
 * After p synchronous sweeps every block of depth <= p holds its fixed-point value.
 * Returns D = max depth (0 for an empty matrix).
 */
int oracle_depth(int n, const int *rowptr, const int *colidx, int *depth) {
    int D = 0;
    for (int i = 0; i < n; ++i)
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int j = colidx[e];
            int lim = i < j ? i : j;
            int d = 0;
            for (long f = rowptr[i]; f < rowptr[i + 1]; ++f) {
                int k = colidx[f];
                if (k >= lim) continue;
                long g = find_block(rowptr, colidx, k, j);
                if (g < 0) continue;
                if (depth[f] > d) d = depth[f];
                if (depth[g] > d) d = depth[g];
            }
            if (i > j) {
                long g = find_block(rowptr, colidx, j, j);
                if (depth[g] > d) d = depth[g];
            }
            depth[e] = d + 1;
            if (depth[e] > D) D = depth[e];
        }
    return D;
}

/* Levels of the block triangular Jacobi iterations (Theorem 3): the lower level of row i is
 * 1 + max over j < i in row i, the upper level 1 + max over j > i. A forward (backward) Jacobi
 * solve is exact after as many sweeps as there are lower (upper) levels. */
void oracle_levels(int n, const int *rowptr, const int *colidx, int *lev_lower, int *lev_upper,
                   int *nlevels_lower, int *nlevels_upper) {
    int nl = 0, nu = 0;
    for (int i = 0; i < n; ++i) {
        int m = 0;
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (colidx[e] < i && lev_lower[colidx[e]] > m) m = lev_lower[colidx[e]];
        lev_lower[i] = m + 1;
        if (lev_lower[i] > nl) nl = lev_lower[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        int m = 0;
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (colidx[e] > i && lev_upper[colidx[e]] > m) m = lev_upper[colidx[e]];
        lev_upper[i] = m + 1;
        if (lev_upper[i] > nu) nu = lev_upper[i];
    }
    *nlevels_lower = nl;
    *nlevels_upper = nu;
}

/* ------------------------------------------------------------------ factorisation */

/*
 * Sequential block ILU(0): the fixed point of h reached by forward substitution in the block
 * Gaussian-elimination (row-major) ordering (Theorem 7), i.e. traditional block ILU(0).
 * For i ascending, for (i,j) in row i ascending:
 *   T = A_ij - sum_{k in K(i,j)} L_ik U_kj   (ascending k, local accumulator)
 *   L_ij = T U_jj^{-1} if i > j,  U_ij = T if i <= j;  U_ii^{-1} is formed when U_ii is final.
 * Returns flag bits.
 */
unsigned oracle_ilu0_seq(int n, const int *rowptr, const int *colidx, const double *A,
                         double *X, double *Dinv) {
    unsigned flags = 0;
    for (int i = 0; i < n; ++i)
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int j = colidx[e];
            int lim = i < j ? i : j;
            double T[BB];
            memcpy(T, A + e * BB, sizeof T);
            for (long f = rowptr[i]; f < rowptr[i + 1]; ++f) {
                int k = colidx[f];
                if (k >= lim) continue;
                long g = find_block(rowptr, colidx, k, j);
                if (g >= 0) mat_sub_mul(T, X + f * BB, X + g * BB);
            }
            if (i > j) {
                mat_mul(X + e * BB, T, Dinv + (long)j * BB);
            } else {
                memcpy(X + e * BB, T, sizeof T);
                if (i == j) flags |= oracle_inv4(T, Dinv + (long)i * BB);
            }
        }
    return flags;
}

/* H_ij(Xp) for one block, with the diagonal inverses Dp of the same iterate (equation blockH). */
static void apply_h(const int *rowptr, const int *colidx, const double *A, const double *Xp,
                    const double *Dp, int i, long e, double *out) {
    int j = colidx[e];
    int lim = i < j ? i : j;
    double T[BB];
    memcpy(T, A + e * BB, sizeof T);
    for (long f = rowptr[i]; f < rowptr[i + 1]; ++f) {
        int k = colidx[f];
        if (k >= lim) continue;
        long g = find_block(rowptr, colidx, k, j);
        if (g >= 0) mat_sub_mul(T, Xp + f * BB, Xp + g * BB);
    }
    if (i > j) mat_mul(out, T, Dp + (long)j * BB);
    else memcpy(out, T, sizeof T);
}

static unsigned diag_inverses(int n, const int *rowptr, const int *colidx, const double *X,
                              double *D) {
    unsigned flags = 0;
#pragma omp parallel for schedule(dynamic, 384) reduction(| : flags)
    for (int j = 0; j < n; ++j)
        flags |= oracle_inv4(X + find_block(rowptr, colidx, j, j) * BB, D + (long)j * BB);
    return flags;
}

static unsigned nonfinite_flag(long count, const double *v) {
    for (long q = 0; q < count; ++q)
        if (!isfinite(v[q])) return ORACLE_FLAG_NONFINITE;
    return 0;
}

/*
 * Synchronous (Jacobi-type) block ILU sweeps x^{p+1} = h(x^p) (Section 4.2), nsw of them,
 * starting from X0 (NULL: X0 = A, the paper's initial guess). Every block is recomputed from
 * the previous iterate only; the diagonal inverses are those of the previous iterate.
 * On return X = x^{nsw} and Dinv = inverses of its diagonal blocks.
 */
unsigned oracle_factor_sync(int n, const int *rowptr, const int *colidx, const double *A,
                            const double *X0, int nsw, double *X, double *Dinv) {
    long Z = rowptr[n];
    double *Xp = (double *)malloc(sizeof(double) * (Z * BB + 1));
    double *Dp = (double *)malloc(sizeof(double) * ((long)n * BB + 1));
    unsigned flags = 0;
    memcpy(Xp, X0 ? X0 : A, sizeof(double) * Z * BB);
    for (int p = 0; p < nsw; ++p) {
        flags |= diag_inverses(n, rowptr, colidx, Xp, Dp);
#pragma omp parallel for schedule(dynamic, 384)
        for (int i = 0; i < n; ++i)
            for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
                apply_h(rowptr, colidx, A, Xp, Dp, i, e, X + e * BB);
        memcpy(Xp, X, sizeof(double) * Z * BB);
    }
    memcpy(X, Xp, sizeof(double) * Z * BB);
    flags |= diag_inverses(n, rowptr, colidx, X, Dinv);
    flags |= nonfinite_flag(Z * BB, X);
    free(Xp);
    free(Dp);
    return flags;
}

/*
 * In-place sweeps in row-major order by a single worker (nonlinear Gauss-Seidel), nsw of them:
 * the asynchronous iteration of Section 3.3/4.2 when one processing element runs the loop.
 * Each diagonal inverse is refreshed as soon as its block is recomputed. One sweep from A
 * reproduces the sequential block ILU(0).
 */
unsigned oracle_factor_gs(int n, const int *rowptr, const int *colidx, const double *A,
                          const double *X0, int nsw, double *X, double *Dinv) {
    long Z = rowptr[n];
    unsigned flags = 0;
    memcpy(X, X0 ? X0 : A, sizeof(double) * Z * BB);
    for (int j = 0; j < n; ++j)
        flags |= oracle_inv4(X + find_block(rowptr, colidx, j, j) * BB, Dinv + (long)j * BB);
    for (int p = 0; p < nsw; ++p)
        for (int i = 0; i < n; ++i)
            for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                double out[BB];
                apply_h(rowptr, colidx, A, X, Dinv, i, e, out);
                memcpy(X + e * BB, out, sizeof out);
                if (colidx[e] == i) flags |= oracle_inv4(out, Dinv + (long)i * BB);
            }
    flags |= nonfinite_flag(Z * BB, X);
    return flags;
}

/*
 * Chunked sweeps (Section 3.3: each OpenMP chunk of consecutive rows is run by one thread in the
 * row-major order, so within a chunk the blocks are computed in a Gaussian-elimination ordering
 * with respect to the chunk's own blocks). The row loop is cut into chunks of R consecutive block
 * rows; a chunk's rows are processed in ascending order and every block of the chunk sees the
 * values its chunk has already produced in this sweep (its own row's L_ik, the U_kj and U_jj^{-1}
 * of earlier rows of the chunk).
 * Deterministic reading of the reads across chunks: every chunk reads the blocks and diagonal
 * inverses of other chunks from the iterate at the start of the sweep, as if all chunks ran at
 * once. `descending` runs the chunks in the reverse order, which must not change the result.
 * Starts from X0 (NULL: A) with Dinv = inverses of X0's diagonal blocks.
 */
unsigned oracle_factor_chunked(int n, const int *rowptr, const int *colidx, const double *A,
                               const double *X0, int nsw, int R, int descending, double *X,
                               double *Dinv) {
    long Z = rowptr[n];
    int nch = (n + R - 1) / R;
    double *Xo = (double *)malloc(sizeof(double) * (Z * BB + 1));
    double *Do = (double *)malloc(sizeof(double) * ((long)n * BB + 1));
    unsigned flags = 0;
    memcpy(X, X0 ? X0 : A, sizeof(double) * Z * BB);
    for (int j = 0; j < n; ++j)
        flags |= oracle_inv4(X + find_block(rowptr, colidx, j, j) * BB, Dinv + (long)j * BB);
    for (int p = 0; p < nsw; ++p) {
        memcpy(Xo, X, sizeof(double) * Z * BB);
        memcpy(Do, Dinv, sizeof(double) * (long)n * BB);
        for (int q = 0; q < nch; ++q) {
            int c = descending ? nch - 1 - q : q;
            int c0 = c * R, c1 = c0 + R < n ? c0 + R : n;
            for (int i = c0; i < c1; ++i)
                for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                    int j = colidx[e];
                    int lim = i < j ? i : j;
                    double T[BB];
                    memcpy(T, A + e * BB, sizeof T);
                    for (long f = rowptr[i]; f < rowptr[i + 1]; ++f) {
                        int k = colidx[f];
                        if (k >= lim) continue;
                        long g = find_block(rowptr, colidx, k, j);
                        if (g < 0) continue;
                        /* L_ik belongs to row i (this chunk); U_kj to row k */
                        mat_sub_mul(T, X + f * BB, (k >= c0 ? X : Xo) + g * BB);
                    }
                    if (i > j) {
                        mat_mul(X + e * BB, T, (j >= c0 ? Dinv : Do) + (long)j * BB);
                    } else {
                        memcpy(X + e * BB, T, sizeof T);
                        if (i == j) flags |= oracle_inv4(T, Dinv + (long)i * BB);
                    }
                }
        }
    }
    flags |= nonfinite_flag(Z * BB, X);
    free(Xo);
    free(Do);
    return flags;
}

/* ------------------------------------------------------------------ triangular solves */

/* y_i (4-vector) -= B_e * x_j */
static void block_matvec_sub(double *y, const double *Bk, const double *x) {
    for (int r = 0; r < BS; ++r) {
        double s = 0.0;
        for (int c = 0; c < BS; ++c) s += Bk[r * BS + c] * x[c];
        y[r] -= s;
    }
}

static void block_matvec(double *y, const double *Bk, const double *x) {
    for (int r = 0; r < BS; ++r) {
        double s = 0.0;
        for (int c = 0; c < BS; ++c) s += Bk[r * BS + c] * x[c];
        y[r] = s;
    }
}

/*
 * Preconditioner application z = (LU)^{-1} r approximated by Jacobi sweeps on the block
 * triangular systems (Algorithm 5 and its backward analogue, synchronous form):
 *   forward,  L unit block lower: y^s_i = r_i - sum_{j<i} L_ij y^{s-1}_j, y^0 = 0;
 *   backward, U block upper:      z^s_i = U_ii^{-1} (y_i - sum_{j>i} U_ij z^{s-1}_j), z^0 = 0;
 * nsw sweeps each. nsw == 0 means no preconditioning (z = r).
 */
void oracle_apply_sync(int n, const int *rowptr, const int *colidx, const double *X,
                       const double *Dinv, const double *r, double *z, int nsw) {
    long nv = (long)n * BS;
    if (nsw <= 0) { memcpy(z, r, sizeof(double) * nv); return; }
    double *yo = (double *)calloc(nv + 1, sizeof(double));
    double *yn = (double *)calloc(nv + 1, sizeof(double));
    double *zo = (double *)calloc(nv + 1, sizeof(double));
    for (int s = 0; s < nsw; ++s) {
#pragma omp parallel for schedule(dynamic, 384)
        for (int i = 0; i < n; ++i) {
            double acc[BS];
            memcpy(acc, r + (long)i * BS, sizeof acc);
            for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
                if (colidx[e] < i) block_matvec_sub(acc, X + e * BB, yo + (long)colidx[e] * BS);
            memcpy(yn + (long)i * BS, acc, sizeof acc);
        }
        double *t = yo; yo = yn; yn = t;
    }
    for (int s = 0; s < nsw; ++s) {
#pragma omp parallel for schedule(dynamic, 384)
        for (int i = 0; i < n; ++i) {
            double acc[BS];
            memcpy(acc, yo + (long)i * BS, sizeof acc);
            for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
                if (colidx[e] > i) block_matvec_sub(acc, X + e * BB, zo + (long)colidx[e] * BS);
            block_matvec(z + (long)i * BS, Dinv + (long)i * BB, acc);
        }
        memcpy(zo, z, sizeof(double) * nv);
    }
    free(yo); free(yn); free(zo);
}

/*
 * Chunked preconditioner application: the sweeps of oracle_apply_sync with the rows cut into
 * chunks of R consecutive rows, each chunk run in order by one worker (Section 3.3 chunks), so
 * that within a chunk the forward sweep is a forward substitution (ascending rows) and the
 * backward sweep a backward substitution (descending rows); entries of other chunks are read from
 * the previous sweep's vector (y^0 = z^0 = 0). nsw sweeps each; nsw == 0 means z = r.
 */
void oracle_apply_chunked(int n, const int *rowptr, const int *colidx, const double *X,
                          const double *Dinv, const double *r, double *z, int nsw, int R,
                          int descending) {
    long nv = (long)n * BS;
    int nch = (n + R - 1) / R;
    if (nsw <= 0) { memcpy(z, r, sizeof(double) * nv); return; }
    double *y = (double *)calloc(nv + 1, sizeof(double));
    double *yo = (double *)calloc(nv + 1, sizeof(double));
    double *zo = (double *)calloc(nv + 1, sizeof(double));
    for (int s = 0; s < nsw; ++s) {
        memcpy(yo, y, sizeof(double) * nv);
        for (int q = 0; q < nch; ++q) {
            int c = descending ? nch - 1 - q : q;
            int c0 = c * R, c1 = c0 + R < n ? c0 + R : n;
            for (int i = c0; i < c1; ++i) {
                double acc[BS];
                memcpy(acc, r + (long)i * BS, sizeof acc);
                for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                    int j = colidx[e];
                    if (j < i) block_matvec_sub(acc, X + e * BB, (j >= c0 ? y : yo) + (long)j * BS);
                }
                memcpy(y + (long)i * BS, acc, sizeof acc);
            }
        }
    }
    memset(z, 0, sizeof(double) * nv);
    for (int s = 0; s < nsw; ++s) {
        memcpy(zo, z, sizeof(double) * nv);
        for (int q = 0; q < nch; ++q) {
            int c = descending ? nch - 1 - q : q;
            int c0 = c * R, c1 = c0 + R < n ? c0 + R : n;
            for (int i = c1 - 1; i >= c0; --i) {
                double acc[BS];
                memcpy(acc, y + (long)i * BS, sizeof acc);
                for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                    int j = colidx[e];
                    if (j > i) block_matvec_sub(acc, X + e * BB, (j < c1 ? z : zo) + (long)j * BS);
                }
                block_matvec(z + (long)i * BS, Dinv + (long)i * BB, acc);
            }
        }
    }
    free(y); free(yo); free(zo);
}

/*
 * Exact block triangular solves (Algorithm 1 in block form): forward substitution with the
 * unit block lower factor, then backward substitution with U, in sequential order.
 */
void oracle_trisolve_exact(int n, const int *rowptr, const int *colidx, const double *X,
                           const double *Dinv, const double *r, double *z) {
    long nv = (long)n * BS;
    double *y = (double *)malloc(sizeof(double) * (nv + 1));
    for (int i = 0; i < n; ++i) {
        double acc[BS];
        memcpy(acc, r + (long)i * BS, sizeof acc);
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (colidx[e] < i) block_matvec_sub(acc, X + e * BB, y + (long)colidx[e] * BS);
        memcpy(y + (long)i * BS, acc, sizeof acc);
    }
    for (int i = n - 1; i >= 0; --i) {
        double acc[BS];
        memcpy(acc, y + (long)i * BS, sizeof acc);
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (colidx[e] > i) block_matvec_sub(acc, X + e * BB, z + (long)colidx[e] * BS);
        block_matvec(z + (long)i * BS, Dinv + (long)i * BB, acc);
    }
    free(y);
}

/* ------------------------------------------------------------------ SpMV and FGMRES */

/* y = A x for a BSR matrix */
void oracle_spmv(int n, const int *rowptr, const int *colidx, const double *A, const double *x,
                 double *y) {
#pragma omp parallel for schedule(dynamic, 384)
    for (int i = 0; i < n; ++i) {
        double acc[BS] = {0.0, 0.0, 0.0, 0.0};
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const double *Bk = A + e * BB;
            const double *xj = x + (long)colidx[e] * BS;
            for (int r = 0; r < BS; ++r)
                for (int c = 0; c < BS; ++c) acc[r] += Bk[r * BS + c] * xj[c];
        }
        memcpy(y + (long)i * BS, acc, sizeof acc);
    }
}

static double dot(long m, const double *a, const double *b) {
    double s = 0.0;
    for (long q = 0; q < m; ++q) s += a[q] * b[q];
    return s;
}

typedef struct {
    int iters, restarts, converged;
    double rel_true_residual;
} oracle_fgmres_result;

/* preconditioner modes for the oracle FGMRES */
#define ORACLE_PC_EXACT (-1)

/*
 * Restarted flexible GMRES with right preconditioning (Saad's FGMRES; the Krylov solver of
 * Sections 1, 2 and 6). x holds the initial guess on entry. Modified Gram-Schmidt, Givens
 * rotations on the (m+1) x m Hessenberg matrix. Stops when the Givens residual estimate drops
 * to rtol * ||b||_2 or after maxit iterations; x is updated at every cycle end and the true
 * residual b - A x decides convergence. The preconditioner is the synchronous sweep apply with
 * apply_nsw sweeps (0: none, ORACLE_PC_EXACT: exact triangular solves).
 * hist (optional, length maxit + 1) receives the residual estimate relative to ||b||
 * at the start (hist[0]) and after every iteration.
 */
int oracle_fgmres(int n, const int *rowptr, const int *colidx, const double *A, const double *b,
                  double *x, int restart, int maxit, double rtol, const double *X,
                  const double *Dinv, int apply_nsw, oracle_fgmres_result *res, double *hist) {
    long nv = (long)n * BS;
    int m = restart;
    double *V = (double *)calloc((long)(m + 1) * nv + 1, sizeof(double));
    double *Zb = (double *)calloc((long)m * nv + 1, sizeof(double));
    double *w = (double *)calloc(nv + 1, sizeof(double));
    double *H = (double *)calloc((long)(m + 1) * m + 1, sizeof(double)); /* H[row*m + col] */
    double *cs = (double *)calloc(m + 1, sizeof(double));
    double *sn = (double *)calloc(m + 1, sizeof(double));
    double *g = (double *)calloc(m + 2, sizeof(double));
    double *yv = (double *)calloc(m + 1, sizeof(double));
    double bnorm = sqrt(dot(nv, b, b));
    double tol = rtol * (bnorm > 0 ? bnorm : 1.0);
    int iters = 0, restarts = 0, converged = 0;
    double beta;

    oracle_spmv(n, rowptr, colidx, A, x, w);
    for (long q = 0; q < nv; ++q) w[q] = b[q] - w[q];
    beta = sqrt(dot(nv, w, w));
    if (hist) hist[0] = beta / (bnorm > 0 ? bnorm : 1.0);
    if (beta <= tol) converged = 1;

    while (!converged && iters < maxit) {
        for (long q = 0; q < nv; ++q) V[q] = w[q] / beta;
        memset(g, 0, sizeof(double) * (m + 2));
        g[0] = beta;
        int k = 0;
        for (; k < m && iters < maxit; ++k) {
            double *vk = V + (long)k * nv, *zk = Zb + (long)k * nv, *vn = V + (long)(k + 1) * nv;
            if (apply_nsw == ORACLE_PC_EXACT)
                oracle_trisolve_exact(n, rowptr, colidx, X, Dinv, vk, zk);
            else
                oracle_apply_sync(n, rowptr, colidx, X, Dinv, vk, zk, apply_nsw);
            oracle_spmv(n, rowptr, colidx, A, zk, vn);
            for (int q = 0; q <= k; ++q) {               /* modified Gram-Schmidt */
                double h = dot(nv, vn, V + (long)q * nv);
                H[q * m + k] = h;
                for (long t = 0; t < nv; ++t) vn[t] -= h * V[(long)q * nv + t];
            }
            double hn = sqrt(dot(nv, vn, vn));
            H[(k + 1) * m + k] = hn;
            if (hn > 0) for (long t = 0; t < nv; ++t) vn[t] /= hn;
            for (int q = 0; q < k; ++q) {                /* previous rotations */
                double a = H[q * m + k], c = H[(q + 1) * m + k];
                H[q * m + k] = cs[q] * a + sn[q] * c;
                H[(q + 1) * m + k] = -sn[q] * a + cs[q] * c;
            }
            double a = H[k * m + k], c = H[(k + 1) * m + k];
            double rho = sqrt(a * a + c * c);
            cs[k] = rho > 0 ? a / rho : 1.0;
            sn[k] = rho > 0 ? c / rho : 0.0;
            H[k * m + k] = rho;
            H[(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            ++iters;
            if (hist) hist[iters] = fabs(g[k + 1]) / (bnorm > 0 ? bnorm : 1.0);
            if (fabs(g[k + 1]) <= tol || hn == 0.0) { ++k; break; }
        }
        /* least squares: back substitution on the k x k triangle, then x += Z y */
        for (int q = k - 1; q >= 0; --q) {
            double s = g[q];
            for (int t = q + 1; t < k; ++t) s -= H[q * m + t] * yv[t];
            yv[q] = s / H[q * m + q];
        }
        for (int q = 0; q < k; ++q)
            for (long t = 0; t < nv; ++t) x[t] += yv[q] * Zb[(long)q * nv + t];
        oracle_spmv(n, rowptr, colidx, A, x, w);
        for (long q = 0; q < nv; ++q) w[q] = b[q] - w[q];
        beta = sqrt(dot(nv, w, w));
        ++restarts;
        if (beta <= tol) converged = 1;
        if (beta == 0.0) break;
    }
    res->iters = iters;
    res->restarts = restarts;
    res->converged = converged;
    res->rel_true_residual = beta / (bnorm > 0 ? bnorm : 1.0);
    free(V); free(Zb); free(w); free(H); free(cs); free(sn); free(g); free(yv);
    return 0;
}

/* ------------------------------------------------------------------ diagnostics */

/*
 * ILU residual ||P_S(LU - A)||_F / ||P_S A||_F over the block pattern (the nonlinear residual
 * of the factor equations), with (LU)_ij = sum_{k in K(i,j)} L_ik U_kj + (i > j ? L_ij U_jj : U_ij).
 */
double oracle_ilu_residual(int n, const int *rowptr, const int *colidx, const double *A,
                           const double *X) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i)
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int j = colidx[e];
            int lim = i < j ? i : j;
            double P[BB];
            if (i > j) mat_mul(P, X + e * BB, X + find_block(rowptr, colidx, j, j) * BB);
            else memcpy(P, X + e * BB, sizeof P);
            for (long f = rowptr[i]; f < rowptr[i + 1]; ++f) {
                int k = colidx[f];
                if (k >= lim) continue;
                long g = find_block(rowptr, colidx, k, j);
                if (g >= 0) {
                    double Q[BB];
                    mat_mul(Q, X + f * BB, X + g * BB);
                    for (int q = 0; q < BB; ++q) P[q] += Q[q];
                }
            }
            for (int q = 0; q < BB; ++q) {
                double d = P[q] - A[e * BB + q];
                num += d * d;
                den += A[e * BB + q] * A[e * BB + q];
            }
        }
    return den > 0 ? sqrt(num / den) : sqrt(num);
}

/* Fixed-point residual ||x - h(x)||_1 of the factor equations (Section 6 metrics), with h using
 * the inverses of x's own diagonal blocks. */
double oracle_fixed_point_residual(int n, const int *rowptr, const int *colidx, const double *A,
                                   const double *X) {
    double *D = (double *)malloc(sizeof(double) * ((long)n * BB + 1));
    diag_inverses(n, rowptr, colidx, X, D);
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            double out[BB];
            apply_h(rowptr, colidx, A, X, D, i, e, out);
            for (int q = 0; q < BB; ++q) s += fabs(X[e * BB + q] - out[q]);
        }
    free(D);
    return s;
}

/* Max-norm (max absolute scalar row sum) of the Jacobi iteration matrices of the triangular
 * solves (Section 6 metrics): for L with unit diagonal it is ||L_strict||_inf; for U it is
 * ||D^{-1} U_strict||_inf with D the block diagonal of U. */
void oracle_jacobi_norms(int n, const int *rowptr, const int *colidx, const double *X,
                         const double *Dinv, double *normL, double *normU) {
    double mL = 0.0, mU = 0.0;
    for (int i = 0; i < n; ++i) {
        double rl[BS] = {0, 0, 0, 0}, ru[BS] = {0, 0, 0, 0};
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int j = colidx[e];
            if (j < i) {
                for (int r = 0; r < BS; ++r)
                    for (int c = 0; c < BS; ++c) rl[r] += fabs(X[e * BB + r * BS + c]);
            } else if (j > i) {
                double P[BB];
                mat_mul(P, Dinv + (long)i * BB, X + e * BB);
                for (int r = 0; r < BS; ++r)
                    for (int c = 0; c < BS; ++c) ru[r] += fabs(P[r * BS + c]);
            }
        }
        for (int r = 0; r < BS; ++r) {
            if (rl[r] > mL) mL = rl[r];
            if (ru[r] > mU) mU = ru[r];
        }
    }
    *normL = mL;
    *normU = mU;
}

/* Factor errors of the ILU-convergence study (Section 6.2): the largest absolute entry of
 * X - X_ilu over the strictly lower blocks, divided by the largest of X0 - X_ilu over the same
 * blocks (the L error), and likewise over the diagonal and strictly upper blocks (the U error).
 * X, X0 and X_ilu are factors in CSR block order. A zero denominator gives the bare numerator. */
void oracle_factor_error(int n, const int *rowptr, const int *colidx, const double *X,
                         const double *X0, const double *Xilu, double *errL, double *errU) {
    double numL = 0.0, denL = 0.0, numU = 0.0, denU = 0.0;
    for (int i = 0; i < n; ++i)
        for (long e = rowptr[i]; e < rowptr[i + 1]; ++e)
            for (int q = 0; q < BB; ++q) {
                double a = fabs(X[e * BB + q] - Xilu[e * BB + q]);
                double b = fabs(X0[e * BB + q] - Xilu[e * BB + q]);
                if (colidx[e] < i) {
                    if (a > numL) numL = a;
                    if (b > denL) denL = b;
                } else {
                    if (a > numU) numU = a;
                    if (b > denU) denU = b;
                }
            }
    *errL = denL > 0 ? numL / denL : numL;
    *errU = denU > 0 ? numU / denU : numU;
}

/* number of OpenMP threads the parallel loops above use (1 without OpenMP) */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
