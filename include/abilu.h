/*
 * abilu.h - C ABI of libabilu.so: asynchronous block ILU(0) preconditioning of 4x4-block sparse
 * (BSR) Jacobians on one AMD Instinct MI355X (gfx950), inside restarted FGMRES.
 *
 * Method: Kashi & Nadarajah, "An asynchronous incomplete block LU preconditioner for
 * computational fluid dynamics on unstructured grids", arXiv:1912.00539.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrix: BSR with block size b = 4 (the d+2 conserved variables of a 2-D cell, Section 2).
 *    rowptr int32[N+1] (rowptr[0] = 0), colidx int32[Z] strictly ascending within each row,
 *    every diagonal block present. Values double[Z][4][4], each block contiguous and row-major.
 *    Vectors double[4N], the 4 unknowns of a cell consecutive.
 *  - Factor: LU[Z][4][4] holds one block per block of A's pattern (ILU(0), Section 6): L_ij for
 *    i > j (L has an implicit identity block diagonal) and U_ij for i <= j, stored in the factor
 *    layout [strictly lower blocks (Z_L) | diagonal blocks U_ii (N) | strictly upper blocks (Z_U)],
 *    each part in row order (columns ascending within a row). The forward and backward sweeps
 *    then read one contiguous part each. abilu_factor_to_csr / abilu_factor_from_csr convert to
 *    and from A's CSR order. Dinv[N][4][4] holds U_ii^{-1}. Element type double (ABILU_F64) or
 *    float (ABILU_F32).
 *  - Memory: every pointer named d_* is device memory on the current HIP device, allocated and
 *    owned by the caller. The library owns only the pattern object (device arrays plus a small
 *    pinned host buffer); the compute entry points allocate nothing. Scratch space is a
 *    caller-provided workspace of at least abilu_workspace_bytes() bytes, 256-byte aligned.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream). Every call is ordered on it.
 *    Only abilu_build_pattern, fgmres_solve, abilu_ilu_residual, abilu_read_flags and
 *    abilu_profile_report block, and they wait on `stream` only.
 *  - Errors: the return value is an abilu_status; negative = error (nothing was launched unless
 *    stated), positive = warning. Nothing throws or aborts across the ABI. Device-side events
 *    (a singular diagonal block replaced, a non-finite value) set bits of a flag word in the
 *    workspace; they are returned by the next blocking call on that workspace (fgmres_solve,
 *    abilu_read_flags).
 *  - Calls that share a workspace or a pattern's pinned buffer must not run concurrently.
 */
#ifndef ABILU_H
#define ABILU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ABILU_OK = 0,
    ABILU_WARN_MODIFIED = 1,   /* a singular diagonal block was replaced by I (modified iteration) */
    ABILU_WARN_NOCONV = 2,     /* FGMRES stopped at maxit without reaching rtol */
    ABILU_EINVAL = -1,         /* bad argument (null pointer, size, enum, workspace too small) */
    ABILU_EPATTERN = -2,       /* unsorted columns, missing diagonal, index out of range */
    ABILU_ENOMEM = -3,         /* device or pinned allocation failed (pattern build only) */
    ABILU_EDEVICE = -4,        /* a HIP runtime call or kernel launch failed */
    ABILU_ENONFINITE = -5      /* a non-finite value appeared (FGMRES result) */
} abilu_status;

/* ABILU_ASYNC_SERIAL: the asynchronous in-place iteration run by a single worker (one quad of
 * lanes) over the block rows in order; the reference schedule with which the paper identifies
 * the asynchronous iteration on one thread with the sequential algorithm (Sections 3.3, 4.2): a
 * factor sweep is then a Gauss-Seidel sweep (from X0 = A, one sweep gives the exact ILU(0)), a
 * forward apply sweep is forward substitution and a backward sweep (rows in descending order)
 * back substitution. It occupies one compute unit lane group: for verification, not speed.
 *
 * ABILU_CHUNK_SYNC, ABILU_CHUNK_ASYNC: the schedule of the paper's implementation (Section 3.3),
 * where the row loop is cut into chunks of consecutive rows and a worker runs a whole chunk in
 * row-major order, so that inside a chunk the factor sweep is a Gauss-Seidel sweep (each block
 * sees the values its chunk has already computed in the sweep), the forward apply sweep a forward
 * substitution and the backward apply sweep (rows descending) a backward substitution. A chunk is
 * run either by a workgroup, its rows grouped by dependence level with a barrier between levels,
 * or by one quad row after row (abilu_chunk_runner); both give exactly the values of the row-major
 * order. Needs the pattern's chunk schedule (abilu_pattern_set_chunks). The iteration is exact after as many sweeps as there are chunks
 * (Section 4.2).
 *   ABILU_CHUNK_SYNC : rows of other chunks are read from the previous sweep (deterministic).
 *   ABILU_CHUNK_ASYNC: in place; rows of other chunks are read as they are in memory.
 * Every apply sweep is launched (no closed-form first sweep). Not accepted by the server. */
typedef enum {
    ABILU_SYNC = 0,
    ABILU_ASYNC = 1,
    ABILU_ASYNC_SERIAL = 2,
    ABILU_CHUNK_SYNC = 3,
    ABILU_CHUNK_ASYNC = 4
} abilu_mode;
typedef enum { ABILU_F64 = 0, ABILU_F32 = 1 } abilu_prec;
typedef enum { ABILU_INIT_FROM_A = 0, ABILU_INIT_FROM_LU = 1 } abilu_init;

/* device flag word bits */
#define ABILU_FLAG_MODIFIED 1u
#define ABILU_FLAG_NONFINITE 2u

typedef struct abilu_pattern abilu_pattern;

/*
 * Analyse a block pattern S_B (Section 4.2) on the device: validate it, locate the diagonal
 * blocks, and build for every block (i,j) the update set of the block ILU equations (equation
 * bilu), K(i,j) = { k < min(i,j) : (i,k) in S_B, (k,j) in S_B }, as a CSR list of position
 * pairs (pos(i,k), pos(k,j)) ascending in k.
 *   nbrows     N block rows (cells), 0 <= N < 2^31 - 1 (so that N + 1 fits in int32)
 *   d_rowptr   device int32[N+1]; d_colidx device int32[Z] (copied; caller keeps ownership)
 *   bs         block size, must be 4
 *   out        receives the pattern handle (release with abilu_pattern_destroy)
 * Blocks on `stream`. Errors: ABILU_EINVAL (bs != 4, N out of range, null pointers), ABILU_EPATTERN
 * (invalid pattern; *out is left NULL), ABILU_ENOMEM, ABILU_EDEVICE.
 */
abilu_status abilu_build_pattern(int32_t nbrows, const int32_t *d_rowptr, const int32_t *d_colidx,
                                 int32_t bs, void *stream, abilu_pattern **out);

/* Free a pattern (NULL is accepted). Not ordered on any stream: the caller must have finished
 * all work that uses it. */
abilu_status abilu_pattern_destroy(abilu_pattern *p);

/* Sizes of a pattern: block rows N, block nonzeros Z, total length of the update-set lists, and
 * the dependency figures of abilu_pattern_depth: the depth D, the number of levels of the strictly
 * lower and strictly upper triangle (each -1 until abilu_pattern_depth has computed them). Any
 * output pointer may be NULL. Non-blocking (reads host fields only). */
abilu_status abilu_pattern_info(const abilu_pattern *p, int32_t *nbrows, int64_t *nnzb, int64_t *npairs,
                                int32_t *depth_D, int32_t *levels_lower, int32_t *levels_upper);

/*
 * Dependency analysis of the block ILU fixed-point problem on the device.
 *  - Depth (Lemma 2 and Theorem 8, Section 4.2): in the Gaussian-elimination ordering of the
 *    blocks the fixed-point map h is strictly lower triangular; block (i,j) reads X_ik and X_kj for
 *    k in K(i,j), and X_jj when i > j. depth(i,j) = 1 + the largest depth of what it reads (1 if
 *    nothing). After p synchronous sweeps every block of depth <= p holds its fixed-point value, so
 *    the sweeps are exact after D = max depth sweeps.
 *  - Levels (Theorem 3, Section 4.1): the lower level of row i is 1 + the largest lower level of
 *    its strictly lower neighbours j < i (1 if none), the upper level likewise over j > i. A
 *    forward (backward) Jacobi sweep solve is exact after as many sweeps as there are lower (upper)
 *    levels.
 * Computed by monotone relaxation passes over all blocks and rows in place (every value starts
 * below its fixed point and only grows towards it), until a pass changes nothing; the result is
 * exact whatever order the passes' reads see. The three counts are kept in the pattern (returned by
 * abilu_pattern_info afterwards).
 *   d_depth         device int32[Z]: depth of every block in CSR order (may be NULL)
 *   d_level_lower   device int32[N]: lower level of every row (may be NULL)
 *   d_level_upper   device int32[N]: upper level of every row (may be NULL)
 *   depth_D, levels_lower, levels_upper: host outputs (may be NULL); D = 0 and no levels for N = 0
 * Allocates and frees temporary device memory (a set-up call, like abilu_build_pattern); no work
 * that uses the pattern may be in flight. Blocks on `stream`. Errors: ABILU_EINVAL, ABILU_ENOMEM,
 * ABILU_EDEVICE.
 */
abilu_status abilu_pattern_depth(abilu_pattern *p, int32_t *d_depth, int32_t *d_level_lower,
                                 int32_t *d_level_upper, int32_t *depth_D, int32_t *levels_lower,
                                 int32_t *levels_upper, void *stream);

/* Copy the pattern's analysis to caller device buffers (for verification): d_diag_pos int32[N],
 * d_pair_ptr int32[Z+1], d_pik int32[npairs], d_pkj int32[npairs]. Any pointer may be NULL. */
abilu_status abilu_pattern_export(const abilu_pattern *p, int32_t *d_diag_pos, int32_t *d_pair_ptr,
                                  int32_t *d_pik, int32_t *d_pkj, void *stream);

/*
 * Build the chunk schedule used by the ABILU_CHUNK_* modes (the chunks of Section 3.3): block rows
 * are cut into chunks of rows_per_chunk consecutive rows (the last one may be shorter). For each
 * chunk the rows are grouped by level in the chunk's lower dependence graph (level 1: no strictly
 * lower neighbour inside the chunk; otherwise one more than the largest level of its strictly
 * lower neighbours inside the chunk), ascending row within a level; likewise by the strictly upper
 * neighbours for the backward apply sweep. Replaces a previous schedule; the pattern owns the
 * device memory (released by abilu_pattern_destroy). No work that uses the pattern may be in
 * flight.
 *   rows_per_chunk  1 .. 4096
 *   runner          abilu_chunk_runner (below)
 * Blocks on `stream`. Errors: ABILU_EINVAL (null pattern, rows_per_chunk or runner out of range),
 * ABILU_ENOMEM, ABILU_EDEVICE (the pattern is then left with no schedule).
 */
abilu_status abilu_pattern_set_chunks(abilu_pattern *p, int32_t rows_per_chunk, int32_t runner,
                                      void *stream);

/* How the chunked sweeps run a chunk (both give the same values):
 *   ABILU_CHUNK_BY_LEVELS: one workgroup per chunk, the rows of each dependence level in
 *                          parallel (one quad per row), a workgroup barrier between levels;
 *   ABILU_CHUNK_BY_ROWS  : one quad per chunk, the chunk's rows in order, no barrier (the
 *                          worker-per-chunk form; fits chunks whose rows form chains). The
 *                          schedule then also holds a 96-byte record per row (its offsets,
 *                          columns, update pairs and where each operand comes from), read one
 *                          row ahead by the sweeps;
 *   ABILU_CHUNK_AUTO     : BY_ROWS when the chunks average fewer than 4 rows per level, else
 *                          BY_LEVELS. */
typedef enum { ABILU_CHUNK_AUTO = 0, ABILU_CHUNK_BY_LEVELS = 1, ABILU_CHUNK_BY_ROWS = 2 } abilu_chunk_runner;

/* Chunk schedule sizes: rows per chunk (0: none built), number of chunks, the runner in use
 * (ABILU_CHUNK_BY_LEVELS or ABILU_CHUNK_BY_ROWS), the largest number of levels in one chunk (lower
 * graph, upper graph) and the number of levels summed over the chunks. Any output pointer may be
 * NULL. */
abilu_status abilu_pattern_chunk_info(const abilu_pattern *p, int32_t *rows_per_chunk, int32_t *nchunks,
                                      int32_t *runner, int32_t *max_levels_lower, int32_t *max_levels_upper,
                                      int64_t *levels_lower, int64_t *levels_upper);

/* Copy one chunk schedule (upper = 0: lower graph, used by the factor and forward sweeps;
 * upper = 1: upper graph, backward sweeps) to caller device buffers, for verification:
 *   d_order    int32[N]            rows of each chunk grouped by level
 *   d_lvptr    int32[nchunks+1]    chunk c owns entries [d_lvptr[c], d_lvptr[c+1]) of d_lvstart
 *   d_lvstart  int32[levels+nchunks]  start of each level of the chunk in d_order, then the
 *                                      chunk's end
 * Any pointer may be NULL. ABILU_EINVAL when no schedule is built. Non-blocking. */
abilu_status abilu_pattern_chunk_export(const abilu_pattern *p, int32_t upper, int32_t *d_order,
                                        int32_t *d_lvptr, int32_t *d_lvstart, void *stream);

/*
 * Orderings of mesh cells (Section 5). Host functions on host arrays, run once per mesh before
 * assembly, as the paper reorders the grid in preprocessing. The graph is the block pattern made
 * symmetric, without its diagonal. Deterministic: every tie goes to the lower index.
 *
 * abilu_find_lines: lines of strongly coupled anisotropic cells (Section 5.1), from one coupling
 * weight per block (for example face area over centroid distance; the paper takes them from the
 * cell geometry). With c_ij = w_ij + w_ji, cell i is anisotropic when max_j c_ij / min_j c_ij >=
 * threshold, and (i, j) is a strong link when c_ij >= max_k c_ik / strong_ratio and
 * c_ij >= max_k c_jk / strong_ratio. Seeds are the anisotropic cells in decreasing anisotropy;
 * a line grows from its seed at one end, then at the other, each step to the unassigned
 * anisotropic neighbour with the strongest strong link. A one-cell line is dropped.
 *   h_rowptr int32[N+1], h_colidx int32[Z]   pattern (host)
 *   h_weight double[Z]                        coupling weight of each block (diagonal ignored)
 *   threshold >= 1, strong_ratio >= 1
 *   h_line_of int32[N]   line of each cell, -1 for a cell in no line (written)
 *   h_line_pos int32[N]  position of the cell in its line from 0, -1 outside lines (written)
 *   nlines               number of lines (written)
 * Errors: ABILU_EINVAL (null pointers, threshold or ratio below 1), ABILU_EPATTERN (index out of
 * range).
 */
abilu_status abilu_find_lines(int32_t n, const int32_t *h_rowptr, const int32_t *h_colidx,
                              const double *h_weight, double threshold, double strong_ratio,
                              int32_t *h_line_of, int32_t *h_line_pos, int32_t *nlines);

/* Orderings (Section 5):
 *   ABILU_ORDER_RCM      reverse Cuthill-McKee from a George-Liu pseudo-peripheral node,
 *                        neighbours in increasing degree; each connected component in turn;
 *   ABILU_ORDER_1WD      George's one-way dissection: separator levels of the level structure
 *                        from a pseudo-peripheral node every delta = sqrt((3w + 13)/2) levels
 *                        (w = vertices per level), the parts between them numbered first (each by
 *                        RCM), the separators last;
 *   ABILU_ORDER_LINE     the cells in their order, each line placed whole where its first cell
 *                        comes (Section 5.1);
 *   ABILU_ORDER_LINE_RCM, ABILU_ORDER_LINE_1WD  hybrid line-X (Section 5.2): RCM or 1WD of the
 *                        graph whose vertices are the lines and the isotropic cells, joined when
 *                        any of their cells are neighbours, each vertex expanded into its cells. */
typedef enum {
    ABILU_ORDER_RCM = 0,
    ABILU_ORDER_1WD = 1,
    ABILU_ORDER_LINE = 2,
    ABILU_ORDER_LINE_RCM = 3,
    ABILU_ORDER_LINE_1WD = 4
} abilu_ordering;

/* Compute an ordering: h_new_of_old int32[N] receives the new index of every cell (a
 * permutation). h_line_of / h_line_pos (as written by abilu_find_lines) are required by the line
 * orderings and ignored otherwise. Errors: ABILU_EINVAL (null pointers, bad ordering, inconsistent
 * lines), ABILU_EPATTERN (index out of range). */
abilu_status abilu_order(int32_t n, const int32_t *h_rowptr, const int32_t *h_colidx, const int32_t *h_line_of,
                         const int32_t *h_line_pos, int32_t ordering, int32_t *h_new_of_old);

/* Workspace bytes needed by abilu_factor, abilu_apply, abilu_ilu_residual and, when
 * fgmres_restart > 0, fgmres_solve with that restart length. */
size_t abilu_workspace_bytes(const abilu_pattern *p, abilu_prec prec, int32_t fgmres_restart);

/*
 * Block ILU(0) factorisation by fixed-point sweeps (Section 4.2): every block of L and U is
 * recomputed from equation bilu in each sweep, all blocks at once.
 *   mode ABILU_SYNC : Jacobi-type iteration x^{p+1} = h(x^p) (deterministic; reads only the
 *                     previous iterate, including its diagonal inverses).
 *   mode ABILU_ASYNC: in-place asynchronous iteration (equation async_blockilu_fp): blocks are
 *                     overwritten as soon as they are computed and later updates read whatever
 *                     values are in memory; sums accumulate in registers only; no atomics on
 *                     values. One kernel launch per sweep bounds the delay by one sweep.
 *                     A row's blocks are computed in ascending column order, each reading the
 *                     row's blocks computed before it; the first sweep from A takes every other
 *                     operand (U_kj, the initial inverses) from A itself, so the prior contents
 *                     of d_LU and d_Dinv are never read.
 *   mode ABILU_ASYNC_SERIAL, ABILU_CHUNK_SYNC, ABILU_CHUNK_ASYNC: see abilu_mode (the chunked
 *                     modes need the pattern's chunk schedule, else ABILU_EINVAL).
 *   init  ABILU_INIT_FROM_A : initial guess X0 = A (the paper's choice, Section 6 setup)
 *         ABILU_INIT_FROM_LU: warm start from the values already in d_LU (Section 3.3 notes the
 *                             previous time step's factors may serve as the initial guess)
 *   d_A     double[Z][4][4] (read; rounded to float on load when prec = ABILU_F32)
 *   d_LU    prec[Z][4][4]   (written; read first for INIT_FROM_LU)
 *   d_Dinv  prec[N][4][4]   (written: inverses of the final diagonal blocks U_ii)
 *   nsweeps >= 0 sweeps (0: d_LU = X0, d_Dinv = inverses of X0's diagonal blocks)
 * A diagonal block that is singular (exact zero pivot in Gaussian elimination with partial
 * pivoting) or has a non-finite inverse is replaced by I and ABILU_FLAG_MODIFIED is set in the
 * workspace flag word (modified iteration, Theorem 8); non-finite factor values set
 * ABILU_FLAG_NONFINITE. Non-blocking. Errors: ABILU_EINVAL, ABILU_EDEVICE.
 */
abilu_status abilu_factor(const abilu_pattern *p, const double *d_A, void *d_LU, void *d_Dinv,
                          abilu_prec prec, int32_t nsweeps, abilu_mode mode, abilu_init init,
                          void *d_work, size_t work_bytes, void *stream);

/*
 * Preconditioner application z ~= (LU)^{-1} r by block Jacobi sweeps on the two triangular
 * systems (Algorithm 5 and its backward analogue, Section 4.1), each from a zero initial guess:
 *   forward  y_i <- r_i - sum_{j<i} L_ij y_j                  (L_ii = I)
 *   backward z_i <- U_ii^{-1} (y_i - sum_{j>i} U_ij z_j)
 * nsweeps forward sweeps then nsweeps backward sweeps (nsweeps = 0: z = r, no preconditioning).
 * SYNC sweeps read the previous sweep's vector; ASYNC sweeps update the vector in place. From the
 * zero initial guess the first sweeps are y = r and z = U_ii^{-1} y and are taken in that closed
 * form (not launched) in these two modes. ABILU_ASYNC_SERIAL runs every sweep, forward rows
 * ascending and backward rows descending, from zero vectors. The chunked modes launch every sweep;
 * within a chunk a forward sweep is a forward substitution and a backward sweep a backward
 * substitution, entries of other chunks being those of the previous sweep (CHUNK_SYNC) or in memory
 * (CHUNK_ASYNC), zero in the first sweep.
 *   d_r double[4N] (read), d_z double[4N] (written; must not alias d_r)
 *   intermediate vectors are stored in prec; d_r is rounded to prec on load.
 * Non-blocking. Errors: ABILU_EINVAL, ABILU_EDEVICE.
 */
abilu_status abilu_apply(const abilu_pattern *p, const void *d_LU, const void *d_Dinv,
                         abilu_prec prec, const double *d_r, double *d_z, int32_t nsweeps,
                         abilu_mode mode, void *d_work, size_t work_bytes, void *stream);

/* Device bytes abilu_apply_noalloc may use on each device (64 MiB). */
#define ABILU_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * abilu_apply without a workspace argument and without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. Same arguments (less the workspace), modes and results as abilu_apply; it runs the same
 * kernels, so the deterministic modes give the same bits. Its four intermediate vectors (4N values
 * of the factor precision each, each rounded up to 256 bytes) live in a library-owned device array
 * of ABILU_NOALLOC_SCRATCH_BYTES, one per device, whose address is taken once per device on the
 * first call there and which is held until the process ends. Hence N <= 1,048,576 block rows in
 * ABILU_F32 and N <= 524,288 in ABILU_F64; a larger pattern gets ABILU_EINVAL before anything is
 * launched (abilu_last_error says why). The pattern must belong to the current device (else
 * ABILU_EINVAL). Every call on a device shares that device's array, which keeps the last call's
 * contents: calls that overlap on one device (several streams or threads) race and must be
 * serialised by the caller; no call relies on the array's previous contents (the one-worker mode
 * clears its vectors with a kernel each time). Calls no hipMalloc, hipFree or hipMemset.
 * Non-blocking. Errors: ABILU_EINVAL, ABILU_EDEVICE.
 */
abilu_status abilu_apply_noalloc(const abilu_pattern *p, const void *d_LU, const void *d_Dinv,
                                 abilu_prec prec, const double *d_r, double *d_z, int32_t nsweeps,
                                 abilu_mode mode, void *stream);

/* Permute a factor between the factor layout and A's CSR block order (for inspection, warm
 * starts from external factors, and verification). d_LU and d_csr: prec[Z][4][4], distinct
 * buffers. Non-blocking. */
abilu_status abilu_factor_to_csr(const abilu_pattern *p, abilu_prec prec, const void *d_LU, void *d_csr,
                                 void *stream);
abilu_status abilu_factor_from_csr(const abilu_pattern *p, abilu_prec prec, const void *d_csr, void *d_LU,
                                   void *stream);

/* Block sparse matrix-vector product y = A x in double precision (the Krylov solver's operator,
 * Section 6 setup). d_x and d_y double[4N] must not alias. Non-blocking. */
abilu_status abilu_spmv(const abilu_pattern *p, const double *d_A, const double *d_x, double *d_y,
                        void *stream);

typedef struct {
    int32_t iters;              /* FGMRES iterations (Arnoldi steps) performed */
    int32_t restarts;           /* completed cycles (x updates) */
    int32_t converged;          /* 1 if ||b - A x||_2 <= rtol ||b||_2 at exit */
    uint32_t flags;             /* workspace flag word at exit (ABILU_FLAG_*) */
    int32_t reorth;             /* iterations that needed the second Gram-Schmidt pass */
    double rel_true_residual;   /* ||b - A x||_2 / ||b||_2 at exit (double precision) */
    double rel_estimate;        /* last Givens residual estimate / ||b||_2 */
} abilu_fgmres_result;

/*
 * Restarted flexible GMRES(restart), right-preconditioned by abilu_apply with the given factor
 * (the outer solver of Sections 1 and 6; flexible because asynchronous application may differ
 * between iterations). Arnoldi basis, orthogonalisation (classical Gram-Schmidt with a second
 * pass when the norm drops below 1/sqrt(2) of its value before orthogonalisation), Givens
 * rotations, least-squares update and true residual are all in double precision on the device.
 * Iterations stop when the Givens estimate reaches rtol ||b||_2 or maxit; x is updated at each
 * cycle end and convergence is decided on the true residual.
 *   d_b double[4N]; d_x double[4N] holds x0 on entry and the solution on exit
 *   options  bit ABILU_FGMRES_ZERO_GUESS: x0 = 0 (d_x is not read; the first residual is b, so
 *            no SpMV is spent on it)
 *   restart >= 1, maxit >= 0, rtol >= 0; apply_sweeps / mode / prec as for abilu_apply
 *   work_bytes >= abilu_workspace_bytes(p, prec, restart)
 * Blocks (one host read of a few scalars per iteration). Returns ABILU_OK, ABILU_WARN_NOCONV,
 * ABILU_WARN_MODIFIED (flag set and converged), ABILU_ENONFINITE, ABILU_EINVAL, ABILU_EDEVICE.
 */
#define ABILU_FGMRES_ZERO_GUESS 1u

abilu_status fgmres_solve(const abilu_pattern *p, const double *d_A, const double *d_b, double *d_x,
                          int32_t restart, int32_t maxit, double rtol, const void *d_LU,
                          const void *d_Dinv, abilu_prec prec, int32_t apply_sweeps, abilu_mode mode,
                          uint32_t options, void *d_work, size_t work_bytes, void *stream,
                          abilu_fgmres_result *out);

/*
 * Nonlinear residual of the factor equations on the pattern, ||P_S(LU - A)||_F / ||P_S(A)||_F,
 * with (LU)_ij = sum_{k in K(i,j)} L_ik U_kj + (i > j ? L_ij U_jj : U_ij) (equation bilu; the
 * quality measure the paper reports for asynchronous factors, Section 6). Accumulated in
 * double. Blocks; the result is written to *h_rel (host memory).
 */
abilu_status abilu_ilu_residual(const abilu_pattern *p, const double *d_A, const void *d_LU,
                                abilu_prec prec, void *d_work, size_t work_bytes, double *h_rel,
                                void *stream);

/*
 * Largest entry-wise difference between a factor and a reference factor, both in the factor
 * layout: *h_lower = max |X - Y| over the entries of the strictly lower blocks (L), *h_upper over
 * the diagonal and strictly upper blocks (U). With Y the exact incomplete factors X_ilu, two calls
 * give the factor errors the paper follows against the sweep count (Section 6.2):
 * ||vec(L - L_ilu)||_inf / ||vec(L_0 - L_ilu)||_inf and likewise for U (L_0, U_0 the initial guess,
 * A in the factor layout by abilu_factor_from_csr). A NaN anywhere shows as NaN.
 *   d_X  prec[Z][4][4] (factor layout); d_Y double[Z][4][4] (factor layout)
 * Uses scratch in the workspace (a workspace of either precision: work_bytes >=
 * abilu_workspace_bytes(p, ABILU_F32, 0)); d_X and d_Y must not lie in it. Blocks.
 */
abilu_status abilu_factor_maxdiff(const abilu_pattern *p, abilu_prec prec, const void *d_X, const double *d_Y,
                                  void *d_work, size_t work_bytes, double *h_lower, double *h_upper, void *stream);

/*
 * Max-norms of the Jacobi iteration matrices of the two block triangular solves (Section 6.2:
 * a smaller norm is a more diagonally dominant factor): *h_norm_l = ||L_strict||_inf (L has a unit
 * diagonal) and *h_norm_u = ||D^{-1} U_strict||_inf with D the block diagonal of U (D^{-1} = Dinv),
 * each the largest absolute scalar row sum. Block products in the factor precision, sums in double.
 * A NaN anywhere shows as NaN. d_LU prec (factor layout), d_Dinv prec[N][4][4]. Workspace as for
 * abilu_factor_maxdiff. Blocks.
 */
abilu_status abilu_jacobi_norms(const abilu_pattern *p, abilu_prec prec, const void *d_LU, const void *d_Dinv,
                                void *d_work, size_t work_bytes, double *h_norm_l, double *h_norm_u,
                                void *stream);

/* Read (and if `clear`, reset) the workspace flag word. Blocks on `stream`. */
abilu_status abilu_read_flags(void *d_work, int32_t clear, uint32_t *h_flags, void *stream);

/* Zero the workspace flag word (ordered on `stream`, non-blocking). */
abilu_status abilu_clear_flags(void *d_work, void *stream);

/* STREAM-style copy d_dst[0:bytes) = d_src[0:bytes) with the same launch style as the library's
 * kernels: the achievable-HBM-bandwidth reference the paper's STREAM comparison calls for
 * (Section 6.1). bytes must be a multiple of 16 and both pointers 16-byte aligned. */
abilu_status abilu_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *stream);

/* Per-kernel timing with HIP events recorded on each launch's stream. enable != 0 starts
 * recording (up to max_launches launches; later launches are not timed) and clears old records;
 * enable = 0 stops. abilu_profile_report waits for the recorded events and writes a JSON object
 * {"kernel": [launches, total_ms, algorithmic_bytes], ...} into buf (NUL-terminated, truncated
 * to len). Algorithmic bytes count every array element a launch must read or write once
 * (gathered blocks and vector entries once, as with perfect cache reuse). The recording state
 * is process-wide and not thread-safe: enable, launch and report from one host thread. */
abilu_status abilu_profile_enable(int32_t enable, int32_t max_launches);
abilu_status abilu_profile_report(char *buf, size_t len);

/* Text of the most recent failed HIP call in this thread (empty if none): the call and the
 * runtime's error string. Copies at most len-1 characters and NUL-terminates. */
abilu_status abilu_last_error(char *buf, size_t len);

const char *abilu_status_string(abilu_status s);

#ifdef __cplusplus
}
#endif

#endif /* ABILU_H */
