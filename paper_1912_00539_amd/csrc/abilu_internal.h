// Internal declarations of libabilu (gfx950). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "abilu.h"

struct abilu_pattern {
    int32_t n = 0;            // block rows
    int64_t nnzb = 0;         // Z
    int64_t npairs = 0;       // total length of the update-set lists
    int64_t nnzb_lower = 0;   // strictly lower blocks
    int64_t nnzb_upper = 0;   // strictly upper blocks
    int32_t *rowptr = nullptr;    // device [n+1]
    int32_t *colidx = nullptr;    // device [Z]
    int32_t *diag_pos = nullptr;  // device [n]
    int32_t *pair_ptr = nullptr;  // device [Z+1], indexed by CSR position
    int32_t *pik = nullptr;       // device [npairs] CSR position of (i,k)
    int32_t *pkj = nullptr;       // device [npairs] CSR position of (k,j)
    int32_t *sik = nullptr;       // device [npairs] factor-layout position of (i,k)
    int32_t *skj = nullptr;       // device [npairs] factor-layout position of (k,j)
    // factor layout: [strictly lower blocks | diagonal blocks | strictly upper blocks], each part
    // in row order; lrow/urow are the row offsets inside the lower/upper parts
    int32_t *lrow = nullptr;      // device [n+1]
    int32_t *urow = nullptr;      // device [n+1]
    int32_t *lcol = nullptr;      // device [ZL+1] columns of the lower part (one padding entry)
    int32_t *ucol = nullptr;      // device [ZU+1] columns of the upper part
    double *pinned = nullptr;     // host pinned, 64 doubles, for blocking scalar reads
    bool symmetric = false;       // (i,j) in S_B implies (j,i) in S_B
    int device = 0;
    // chunk schedule (abilu_pattern_set_chunks): chunks of chunk_rows consecutive rows; per chunk,
    // the rows grouped by level in the chunk's lower (forward, factor) and upper (backward)
    // dependence graphs. Schedule s (0 lower, 1 upper): order[s][N] rows, lvptr[s][nchunks+1]
    // offsets into lvstart[s], whose entries for chunk c are the starts (positions in order[s])
    // of its levels followed by the chunk's end.
    int32_t chunk_rows = 0;
    int32_t nchunks = 0;
    int32_t chunk_runner = 0;     // ABILU_CHUNK_BY_LEVELS or ABILU_CHUNK_BY_ROWS (resolved, never AUTO)
    int32_t max_levels[2] = {0, 0};
    int64_t total_levels[2] = {0, 0};
    int32_t *order[2] = {nullptr, nullptr};
    int32_t *lvptr[2] = {nullptr, nullptr};
    int32_t *lvstart[2] = {nullptr, nullptr};
    // per-row records of the quad-per-chunk runner (ABILU_CHUNK_BY_ROWS only): REC_INTS int32 per
    // row in REC_INTS / 4 planes of int4, each step-major (row c * chunk_rows + t at index
    // t * nchunks + c); then 4 ints of per-pattern maxima
    int32_t *rec = nullptr;
    int32_t rec_max[3] = {0, 0, 0};   // largest strictly lower / strictly upper / pair count of a row
    // dependency analysis (abilu_pattern_depth): depth D and the lower/upper level counts, -1 until
    // computed
    int32_t depth_D = -1;
    int32_t levels[2] = {-1, -1};
};

namespace abilu {

constexpr int BS = 4;
constexpr int BB = 16;
constexpr int WG = 256;                 // threads per workgroup (4 wavefronts of 64)
constexpr int ROWS_PER_WG = WG / BS;    // one quad of 4 lanes per block row

// vector kernels: elements per thread and workgroup tile
constexpr int VEC_E = 8;
constexpr int VEC_TILE = WG * VEC_E;    // 2048 doubles per workgroup

__host__ __device__ inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ workspace layout
struct Workspace {
    size_t flags;      // uint32 flag word (in the 256-byte header)
    size_t status;     // double[8] scalars read back by the host (header)
    size_t x2, d2;     // SYNC factor ping-pong buffers (prec)
    size_t ya, yb, za, zb;  // apply vectors (prec)
    size_t partials;   // double[(restart+2) * nb_vec]
    size_t hess;       // double[(restart+1) * restart], column-major, ld = restart+1
    size_t cs, sn, g, coef, misc;  // double[restart+2] each; misc double[16]
    size_t red;        // double[restart+4]: outputs of column reductions
    size_t V, Z;       // double[(restart+1) * 4N], double[restart * 4N]
    size_t total;
    int nb_vec;        // workgroups of the vector kernels
    int restart;
};

Workspace layout(const abilu_pattern *p, abilu_prec prec, int restart);

// ------------------------------------------------------------------ launch helpers
// Per-launch HIP-event timing (abilu_profile_enable). Records around every kernel launch,
// together with the launch's algorithmic bytes (every array element the kernel must touch,
// counted once).
struct ProfScope {
    ProfScope(const char *name, hipStream_t s, double bytes = 0.0);
    ~ProfScope();
    int slot;
    hipStream_t stream;
};
int prof_mark();                          // index of the next profiled launch
void prof_cancel_bytes(int from, int to); // zero the bytes of launches [from, to): skipped work
void prof_add_bytes(int slot, double delta);  // correct the bytes of one profiled launch

abilu_status launch_status();   // hipGetLastError -> status (records the error text)

// Record a failed HIP call (text returned by abilu_last_error); true if e == hipSuccess.
bool hip_ok(hipError_t e, const char *what);
// Record an error text of the library's own (returned by abilu_last_error).
void note_error(const char *what);

// Algorithmic-byte model inputs of a pattern (doubles to avoid overflow in byte formulas).
struct Sizes {
    double N, Z, ZL, ZU, P;
};
inline Sizes sizes(const abilu_pattern *p) {
    return Sizes{(double)p->n, (double)p->nnzb, (double)p->nnzb_lower, (double)p->nnzb_upper, (double)p->npairs};
}

// Algorithmic bytes of one launch (every element touched once; gathered vector entries once).
// forward: lrow, columns and blocks of the strictly lower part, r (f64),
// input vector (element size sY), output vector; EMIT_Z adds Dinv and the z output.
inline double bytes_fwd(const Sizes &z, double sF, double sY, bool emit) {
    double b = 4 * (z.N + 1) + 4 * z.ZL + 16 * sF * z.ZL + 32 * z.N + 4 * z.N * sY + 4 * z.N * sF;
    return emit ? b + 16 * sF * z.N + 4 * z.N * sF : b;
}
// backward: urow, columns and blocks of the strictly upper part, y, z input,
// Dinv, output (element size sZ), optional second output in precision sF
inline double bytes_bwd(const Sizes &z, double sF, double sZ, bool dual) {
    double b = 4 * (z.N + 1) + 4 * z.ZU + 16 * sF * z.ZU + 4 * z.N * sF + 4 * z.N * sF + 16 * sF * z.N + 4 * z.N * sZ;
    return dual ? b + 4 * z.N * sF : b;
}

// Algorithmic bytes of one launch: every array element touched once.
// init with copy: rowptr, diag_pos, lrow, urow, A (f64), X0 written, Dinv written
// init without copy: diag_pos, diagonal blocks of the source, Dinv written
inline double bytes_init(const Sizes &z, double sS, double sF, bool copy) {
    if (copy) return 4 * (z.N + 1) + 12 * z.N + 128 * z.Z + 16 * sF * z.Z + 16 * sF * z.N;
    return 4 * z.N + 16 * sS * z.N + 16 * sF * z.N;
}
// sweep: rowptr, diag_pos, lrow, urow, colidx of strictly lower blocks, pair_ptr at 4 places per
// row, the pair lists, A (f64), the blocks the update sets read from X (min(2P, Z) of them, half
// on each side; none when a side comes from A), Dinv read, X written, Dinv written
inline double bytes_sweep(const Sizes &z, double sF, bool l_from_a, bool u_from_a) {
    const double m = (2 * z.P < z.Z ? 2 * z.P : z.Z) / 2;
    const double xr = (l_from_a ? 0.0 : 16 * sF * m) + (u_from_a ? 0.0 : 16 * sF * m);
    return 4 * (z.N + 1) + 12 * z.N + 4 * z.ZL + 16 * z.N + 8 * z.P + 128 * z.Z + xr + 16 * sF * z.N +
           16 * sF * z.Z + 16 * sF * z.N;
}

// first sweep from A forming the initial inverses itself: as a sweep with U (and, in SYNC, L)
// from A, without the Dinv read (the diagonal blocks it inverts are elements of A, counted once)
inline double bytes_sweep_from_a(const Sizes &z, double sF, bool l_from_a) {
    return bytes_sweep(z, sF, l_from_a, true) - 16 * sF * z.N;
}

// SpMV: rowptr, colidx, A (f64), x gathered once, y written (+ b read when RESID)
inline double bytes_spmv(const Sizes &z, bool resid) {
    return 4 * (z.N + 1) + 4 * z.Z + 128 * z.Z + 32 * z.N + 32 * z.N + (resid ? 32 * z.N : 0.0);
}

// ------------------------------------------------------------------ device prefix sums (scan.hip)
// Tiles needed by scan_exclusive for `len` elements; the `tot` scratch needs scan_tiles(len) + 1
// int64 entries. out64 (optional) gets len + 1 offsets, out32 len + 1 offsets.
int scan_tiles(int64_t len);
hipError_t scan_exclusive(int64_t len, const int64_t *in, int64_t *tot, int64_t *out64, int32_t *out32,
                          hipStream_t s);

// ------------------------------------------------------------------ pattern analysis into caller buffers
// (pattern.hip; used by abilu_build_pattern and by the server, which carves the arrays out of its
// pool). Scratch: pattern_scratch_bytes(n, Z) device bytes, kept between the two stages.
size_t pattern_scratch_bytes(int32_t n, int64_t Z);
// The pattern-analysis scratch of pattern_scratch_bytes(n, Z) bytes: a 256-byte header (the
// validation error word), then int64 cnt[Z + n + 2] (counts to scan), ptr64[Z + n + 2] (int64
// offsets, kept for the fill) and the scan's tile sums. The one definition of these offsets.
struct PatScratch {
    int64_t *cnt, *ptr64, *tot;
};
inline PatScratch pat_scratch(void *scratch, int32_t n, int64_t Z) {
    const int64_t len = Z + n + 2;
    int64_t *cnt = (int64_t *)((char *)scratch + 256);
    return PatScratch{cnt, cnt + len, cnt + 2 * len};
}
abilu_status pattern_validate_async(int32_t n, int64_t Z, const int32_t *rowptr, const int32_t *colidx,
                                    int32_t *diag_pos, void *scratch, unsigned *h_err, hipStream_t s);
abilu_status pattern_count_async(int32_t n, int64_t Z, const int32_t *rowptr, const int32_t *colidx,
                                 const int32_t *diag_pos, int32_t *lrow, int32_t *urow, int32_t *pair_ptr,
                                 void *scratch, int64_t *h_sizes, hipStream_t s);
bool pattern_sizes_ok(int32_t n, int64_t Z, const int64_t *sizes);   // sizes = {ZL, ZU, npairs}
abilu_status pattern_count(int32_t n, int64_t Z, const int32_t *rowptr, const int32_t *colidx, int32_t *diag_pos,
                           int32_t *lrow, int32_t *urow, int32_t *pair_ptr, void *scratch, int64_t *h_pinned,
                           hipStream_t s, int64_t *ZL, int64_t *ZU, int64_t *npairs);
abilu_status pattern_fill(int32_t n, int64_t Z, int64_t ZL, int64_t ZU, int64_t npairs, const int32_t *rowptr,
                          const int32_t *colidx, const int32_t *diag_pos, const int32_t *lrow, const int32_t *urow,
                          int32_t *lcol, int32_t *ucol, int32_t *pik, int32_t *pkj, int32_t *sik, int32_t *skj,
                          const void *scratch, hipStream_t s);

// A mode the single-system entry points accept for this pattern (the chunked modes need the
// pattern's chunk schedule).
inline bool mode_ok(const abilu_pattern *p, abilu_mode m) {
    if (m == ABILU_SYNC || m == ABILU_ASYNC || m == ABILU_ASYNC_SERIAL) return true;
    return (m == ABILU_CHUNK_SYNC || m == ABILU_CHUNK_ASYNC) && p->chunk_rows > 0;
}

// Release a pattern's chunk schedule (chunks.hip).
void free_chunks(abilu_pattern *p);
int32_t chunk_runner_auto(int n, int nch, const int64_t *total_levels);
constexpr int MAX_CHUNK_ROWS = 4096;

// Per-row record of the quad-per-chunk runner: everything a row's chunked sweep needs to find its
// operands, in one 96-byte read, classified by where each operand comes from.
//   [0] rowptr[i]  [1] lrow[i]  [2] urow[i]
//   [3] meta: bits 0-3 min(nl, 15), 4-7 min(nu, 15), 8-11 min(np, 15) (strictly lower blocks,
//       strictly upper blocks, update pairs of the row); bits 12 + 2u: source of the lower
//       neighbour u (u < 4); bits 20 + 2w: source of the upper neighbour w (w < 4)
//   [4..7] columns of the first four strictly lower blocks
//   [8..11] update pair p (p < 4, in pair-list order): bits 0-3 target block (0-3 lower block u,
//       4 diagonal, 5-8 upper block w), 4-5 ordinal of L_ik among the row's lower blocks,
//       6-7 source of U_kj, 8-9 ordinal of U_kj among row i-1's upper blocks (source REC_PREV;
//       meaningful when row i-1 has at most REC_CAP of them)
//   [12..15] factor-layout position of U_kj  [16..19] CSR position of (k, j)
//   [20..23] columns of the first four strictly upper blocks
// A row with more than REC_CAP lower or upper blocks or update pairs takes the general code.
constexpr int REC_INTS = 24;
constexpr int REC_CAP = 4;
// Sources: the neighbouring row of the chunk computed just before (row i - 1 forward, i + 1
// backward), another row of the chunk, a row outside the chunk.
enum : int { REC_PREV = 0, REC_CHUNK = 1, REC_OUT = 2 };

// ------------------------------------------------------------------ entry points used across files
abilu_status apply_impl(const abilu_pattern *p, const void *LU, const void *Dinv, abilu_prec prec,
                        const double *r, double *z, int nsweeps, abilu_mode mode, char *work,
                        const Workspace &W, hipStream_t s);
// Whether the last kernel of apply_impl(nsweeps, mode) ran its workgroups in descending row order.
bool apply_ends_descending(int nsweeps, abilu_mode mode);
// desc: run the workgroups in descending row order (the result does not depend on it; a kernel
// that starts on the rows its predecessor touched last finds them in the Infinity Cache).
abilu_status spmv_impl(const abilu_pattern *p, const double *A, const double *x, double *y,
                       const double *b, bool desc, hipStream_t s);

}  // namespace abilu

// ------------------------------------------------------------------ device helpers
namespace abilu_dev {

// Position in the factor layout of CSR position e of row i (d = diag_pos[i]).
__device__ __forceinline__ int split_pos(int e, int i, int b0, int d, int lbase, int ubase, int ZL, int n) {
    return e < d ? lbase + (e - b0) : (e == d ? ZL + i : ZL + n + ubase + (e - d - 1));
}

// Broadcast lane L of each quad (4 consecutive lanes) to the whole quad with one DPP
// quad_perm move per 32-bit word. All four lanes of the quad must be active.
template <int L>
__device__ __forceinline__ float qb(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), L * 0x55, 0xF, 0xF, false));
}
template <int L>
__device__ __forceinline__ double qb(double v) {
    long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    lo = __builtin_amdgcn_update_dpp(0, lo, L * 0x55, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, L * 0x55, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned long long)(unsigned)lo);
}

// Arithmetic of the block products. In double precision every product is rounded before it is
// added and the terms are added left to right, with no fused multiply-add: the evaluation of a
// plain loop over the terms, so that each double-precision result is reproducible operation for
// operation. In single precision the compiler fuses products into the sums.
template <typename T>
__device__ __forceinline__ T dot4(T a0, T b0, T a1, T b1, T a2, T b2, T a3, T b3) {
    if constexpr (sizeof(T) == 8) {
#pragma clang fp contract(off)
        return ((a0 * b0 + a1 * b1) + a2 * b2) + a3 * b3;
    } else {
        return a0 * b0 + a1 * b1 + a2 * b2 + a3 * b3;
    }
}

// a - b c (the product rounded first in double precision).
template <typename T>
__device__ __forceinline__ T sub_prod(T a, T b, T c) {
    if constexpr (sizeof(T) == 8) {
#pragma clang fp contract(off)
        return a - b * c;
    } else {
        return a - b * c;
    }
}

// Row r (this lane's row) of a 4x4 block at `blk` (row-major), converted to T.
template <typename T, typename S>
__device__ __forceinline__ void load_row(const S *blk, int r, T (&v)[4]) {
    const S *p = blk + r * 4;
    if constexpr (sizeof(S) == 4) {
        float4 q = *reinterpret_cast<const float4 *>(p);
        v[0] = (T)q.x; v[1] = (T)q.y; v[2] = (T)q.z; v[3] = (T)q.w;
    } else {
        double2 a = *reinterpret_cast<const double2 *>(p);
        double2 b = *reinterpret_cast<const double2 *>(p + 2);
        v[0] = (T)a.x; v[1] = (T)a.y; v[2] = (T)b.x; v[3] = (T)b.y;
    }
}

template <typename T>
__device__ __forceinline__ void store_row(T *blk, int r, const T (&v)[4]) {
    T *p = blk + r * 4;
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2 *>(p + 2) = make_double2(v[2], v[3]);
    }
}

// Full 4x4 block assembled in every lane of the quad from the lanes' rows.
template <typename T>
__device__ __forceinline__ void gather_block(const T (&row)[4], T (&M)[16]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        M[0 * 4 + c] = qb<0>(row[c]);
        M[1 * 4 + c] = qb<1>(row[c]);
        M[2 * 4 + c] = qb<2>(row[c]);
        M[3 * 4 + c] = qb<3>(row[c]);
    }
}

// out[c] = sum_m a[m] * B[m][c], where this lane holds row a of the left factor and row r of B;
// rows m of B come from the quad's lanes by DPP broadcast.
template <typename T>
__device__ __forceinline__ void row_times_block(const T (&a)[4], const T (&brow)[4], T (&out)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        T b0 = qb<0>(brow[c]), b1 = qb<1>(brow[c]), b2 = qb<2>(brow[c]), b3 = qb<3>(brow[c]);
        out[c] = dot4(a[0], b0, a[1], b1, a[2], b2, a[3], b3);
    }
}

// acc[c] -= sum_m a[m] * B[m][c]
template <typename T>
__device__ __forceinline__ void row_times_block_sub(const T (&a)[4], const T (&brow)[4], T (&acc)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        T b0 = qb<0>(brow[c]), b1 = qb<1>(brow[c]), b2 = qb<2>(brow[c]), b3 = qb<3>(brow[c]);
        acc[c] -= dot4(a[0], b0, a[1], b1, a[2], b2, a[3], b3);
    }
}

// The 4-vector held one element per lane of the quad, broadcast to every lane.
template <typename T>
__device__ __forceinline__ void gather_vec(T v, T (&x)[4]) {
    x[0] = qb<0>(v); x[1] = qb<1>(v); x[2] = qb<2>(v); x[3] = qb<3>(v);
}

// Row r (this lane's index in the quad) of the inverse of the 4x4 block M, which every lane of
// the quad holds: Gaussian elimination with partial pivoting and back substitution, all indices
// static (row exchanges are selects). Every lane eliminates on M but carries only column r of
// the identity as right-hand side and back-substitutes only column r of the inverse; the quad
// then exchanges columns for rows by DPP. Each element goes through the same operations, in the
// same order, as in the elimination on the full [M | I] (10 instead of 22 divisions per lane).
// Returns false for the whole quad, with the identity row, if a pivot is exactly zero or any
// element of the inverse is not finite (the modified iteration's replacement).
template <typename T>
__device__ __forceinline__ bool inv4_row(T (&M)[16], int r, T (&out)[4]) {
    T x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = (q == r) ? T(1) : T(0);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int p = k;
        T best = fabs(M[k * 4 + k]);
#pragma unroll
        for (int q = k + 1; q < 4; ++q) {
            T a = fabs(M[q * 4 + k]);
            bool gt = a > best;
            best = gt ? a : best;
            p = gt ? q : p;
        }
#pragma unroll
        for (int q = k + 1; q < 4; ++q) {
            bool s = (p == q);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                T a = M[k * 4 + c], b = M[q * 4 + c];
                M[k * 4 + c] = s ? b : a;
                M[q * 4 + c] = s ? a : b;
            }
            T u = x[k], v = x[q];
            x[k] = s ? v : u;
            x[q] = s ? u : v;
        }
        T piv = M[k * 4 + k];
        ok = ok && (piv != T(0));
#pragma unroll
        for (int q = k + 1; q < 4; ++q) {
            T f = M[q * 4 + k] / piv;
#pragma unroll
            for (int c = 0; c < 4; ++c) M[q * 4 + c] = sub_prod(M[q * 4 + c], f, M[k * 4 + c]);
            x[q] = sub_prod(x[q], f, x[k]);
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        T s = x[k];
#pragma unroll
        for (int m = k + 1; m < 4; ++m) s = sub_prod(s, M[k * 4 + m], x[m]);
        x[k] = s / M[k * 4 + k];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) ok = ok && isfinite(x[q]);
    // the block is replaced if any lane's column failed
    const int okl = ok ? 1 : 0;
    const int okq = __builtin_amdgcn_update_dpp(0, okl, 0x00, 0xF, 0xF, false) &
                    __builtin_amdgcn_update_dpp(0, okl, 0x55, 0xF, 0xF, false) &
                    __builtin_amdgcn_update_dpp(0, okl, 0xAA, 0xF, 0xF, false) &
                    __builtin_amdgcn_update_dpp(0, okl, 0xFF, 0xF, 0xF, false);
    // out[c] = inverse(r, c) = element r of lane c's column
    const bool b0 = (r & 1) != 0, b1 = (r & 2) != 0;
    T col[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c == 0) { col[0] = qb<0>(x[0]); col[1] = qb<0>(x[1]); col[2] = qb<0>(x[2]); col[3] = qb<0>(x[3]); }
        if (c == 1) { col[0] = qb<1>(x[0]); col[1] = qb<1>(x[1]); col[2] = qb<1>(x[2]); col[3] = qb<1>(x[3]); }
        if (c == 2) { col[0] = qb<2>(x[0]); col[1] = qb<2>(x[1]); col[2] = qb<2>(x[2]); col[3] = qb<2>(x[3]); }
        if (c == 3) { col[0] = qb<3>(x[0]); col[1] = qb<3>(x[1]); col[2] = qb<3>(x[2]); col[3] = qb<3>(x[3]); }
        const T lo = b0 ? col[1] : col[0];
        const T hi = b0 ? col[3] : col[2];
        out[c] = okq ? (b1 ? hi : lo) : ((c == r) ? T(1) : T(0));
    }
    return okq != 0;
}

template <typename T>
__device__ __forceinline__ unsigned nonfinite4(const T (&v)[4]) {
    return (isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(v[3])) ? 0u : ABILU_FLAG_NONFINITE;
}

}  // namespace abilu_dev
