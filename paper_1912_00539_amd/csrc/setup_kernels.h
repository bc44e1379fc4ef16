// Device bodies of the setup kernels: prefix scans, pattern analysis and the seeded request
// generator. Each body takes its tile index `blk` explicitly, so the single-system kernels and
// the server's batched admission kernels (one launch over the tiles of many requests) share them.
#pragma once

#include <climits>
#include <cmath>

#include "abilu_gen.h"
#include "abilu_internal.h"

namespace abilu_setup {

using namespace abilu;
using namespace abilu_dev;

// ------------------------------------------------------------------ exclusive prefix sums
// Three phases over int64 counts: the sum of each tile (SCAN_T threads, SCAN_TILE elements), an
// exclusive scan of the tile sums in one workgroup, then each tile scanned again from its offset
// and written as len + 1 offsets. The counts are read twice and only the offsets are written: no
// intermediate array goes to memory and back.
constexpr int SCAN_T = 256, SCAN_E = 8, SCAN_TILE = SCAN_T * SCAN_E;

__device__ __forceinline__ long long block_exclusive(long long v, long long *sh, long long *total) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        long long a = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    long long inc = sh[t];
    *total = sh[SCAN_T - 1];
    __syncthreads();
    return inc - v;
}

// tot[blk] = sum of the tile's counts (read strided, so each load instruction is coalesced)
__device__ __forceinline__ void scan_reduce_body(int blk, int64_t len, const int64_t *__restrict__ in,
                                                 int64_t *__restrict__ tot) {
    __shared__ long long sh[SCAN_T];
    const int64_t first = (int64_t)blk * SCAN_TILE;
    long long s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_E; ++q) {
        const int64_t e = first + (int64_t)q * SCAN_T + threadIdx.x;
        if (e < len) s += in[e];
    }
    long long total;
    (void)block_exclusive(s, sh, &total);
    if (threadIdx.x == 0) tot[blk] = total;
}

__device__ __forceinline__ void scan_totals_body(int ntiles, int64_t *__restrict__ tot,
                                                        int64_t *__restrict__ grand) {
    __shared__ long long sh[SCAN_T];
    long long carry = 0;
    for (int base = 0; base < ntiles; base += SCAN_T) {
        int q = base + threadIdx.x;
        long long v = (q < ntiles) ? tot[q] : 0;
        long long total;
        long long pre = block_exclusive(v, sh, &total);
        if (q < ntiles) tot[q] = carry + pre;
        carry += total;
    }
    if (threadIdx.x == 0) *grand = carry;
}

// One tile per workgroup, SCAN_E consecutive counts per thread: offsets out[e] = tot[blk] + the
// tile's exclusive sum before e, for e < len; the workgroup holding index len writes the grand
// total there (a workgroup past the last full tile exists for that alone).
__device__ __forceinline__ void scan_finish_body(int blk, int64_t len, const int64_t *__restrict__ in,
                                                 const int64_t *__restrict__ tot, const int64_t *__restrict__ grand,
                                                 int64_t *__restrict__ ptr64, int32_t *__restrict__ ptr32) {
    __shared__ long long sh[SCAN_T];
    const int64_t first = (int64_t)blk * SCAN_TILE;
    const int64_t base = first + (int64_t)threadIdx.x * SCAN_E;
    long long v[SCAN_E], s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_E; ++q) {
        v[q] = (base + q < len) ? in[base + q] : 0;
        s += v[q];
    }
    long long total;
    long long pre = block_exclusive(s, sh, &total) + (first < len ? tot[blk] : 0);
#pragma unroll
    for (int q = 0; q < SCAN_E; ++q) {
        const int64_t e = base + q;
        if (e < len) {
            if (ptr64) ptr64[e] = pre;
            ptr32[e] = (int32_t)pre;
            pre += v[q];
        } else if (e == len) {
            if (ptr64) ptr64[len] = *grand;
            ptr32[len] = (int32_t)*grand;
        }
    }
}


// ------------------------------------------------------------------ pattern analysis
// position of column j in row k, or -1 (binary search over the sorted row)
__device__ __forceinline__ int find_col(const int32_t *rowptr, const int32_t *colidx, int k, int j) {
    int lo = rowptr[k], hi = rowptr[k + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int c = colidx[mid];
        if (c == j) return mid;
        if (c < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

__device__ __forceinline__ void pat_rows_body(int blk, int n, int64_t Z, const int32_t *__restrict__ rowptr,
                           const int32_t *__restrict__ colidx, int32_t *__restrict__ diag_pos,
                           unsigned *__restrict__ err) {
    int i = blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b0 = rowptr[i], b1 = rowptr[i + 1];
    bool bad = (b0 < 0) || (b1 < b0) || ((int64_t)b1 > Z);
    int d = -1;
    if (!bad) {
        int prev = -1;
        for (int e = b0; e < b1; ++e) {
            int j = colidx[e];
            if (j < 0 || j >= n || j <= prev) { bad = true; break; }
            prev = j;
            if (j == i) d = e;
        }
    }
    if (d < 0) bad = true;
    diag_pos[i] = d;
    if (bad) atomicOr(err, 1u);
}

// position of column j in the strictly upper part of row k (j > k), or -1 (binary search)
__device__ __forceinline__ int find_upper(const int32_t *rowptr, const int32_t *colidx, const int32_t *diag_pos,
                                          int k, int j) {
    int lo = diag_pos[k] + 1, hi = rowptr[k + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int c = colidx[mid];
        if (c == j) return mid;
        if (c < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// The count and fill bodies run one thread per block row, PAT_ROWS rows per workgroup. A
// workgroup's outputs form one contiguous range; when it holds at most PAT_STAGE entries they are
// staged in LDS and written together, so every line is written whole (a thread's own entries are
// a few words at a row's stride, which partly written lines would write back several times).
constexpr int PAT_ROWS = 128;
constexpr int PAT_STAGE = 1024;

// |K(i,j)| for every block (i,j) of the row: the k < min(i,j) of the row's strictly lower blocks
// with (k,j) in S_B (an upper block of row k, since k < j)
__device__ __forceinline__ void pat_count_body(int blk, int n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ colidx,
                                               const int32_t *__restrict__ diag_pos, int64_t *__restrict__ cnt) {
    __shared__ int32_t sh[PAT_STAGE];
    const int i0 = blk * PAT_ROWS;
    if (i0 >= n) return;   // the whole workgroup
    const int i1 = min(n, i0 + PAT_ROWS);
    const int base = rowptr[i0], len = rowptr[i1] - base;
    const bool staged = len <= PAT_STAGE;
    const int i = i0 + (int)threadIdx.x;
    if (i < i1) {
        const int b0 = rowptr[i], b1 = rowptr[i + 1];
        for (int e = b0; e < b1; ++e) {
            const int j = colidx[e];
            const int lim = i < j ? i : j;
            int c = 0;
            for (int f = b0; f < b1; ++f) {
                const int k = colidx[f];
                if (k >= lim) break;
                c += (find_upper(rowptr, colidx, diag_pos, k, j) >= 0);
            }
            if (staged) sh[e - base] = c;
            else cnt[e] = c;
        }
    }
    __syncthreads();
    if (staged)
        for (int t = threadIdx.x; t < len; t += blockDim.x) cnt[base + t] = sh[t];
}

// The update-set lists: for block e = (i,j), entries ptr[e] .. ptr[e+1] hold, ascending in k, the
// CSR positions of (i,k) and (k,j) and their factor-layout positions ((i,k) is strictly lower in
// row i, (k,j) strictly upper in row k).
__device__ __forceinline__ void pat_fill_body(int blk, int n, int ZL, const int32_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ colidx,
                                              const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow,
                                              const int32_t *__restrict__ urow, const int64_t *__restrict__ ptr,
                                              int32_t *__restrict__ pik, int32_t *__restrict__ pkj,
                                              int32_t *__restrict__ sik, int32_t *__restrict__ skj) {
    __shared__ int32_t sh[4][PAT_STAGE];
    const int i0 = blk * PAT_ROWS;
    if (i0 >= n) return;   // the whole workgroup
    const int i1 = min(n, i0 + PAT_ROWS);
    const int64_t pbase = ptr[rowptr[i0]], plen = ptr[rowptr[i1]] - pbase;
    const bool staged = plen <= PAT_STAGE;
    const int i = i0 + (int)threadIdx.x;
    if (i < i1) {
        const int b0 = rowptr[i], b1 = rowptr[i + 1], lb = lrow[i];
        for (int e = b0; e < b1; ++e) {
            const int j = colidx[e];
            const int lim = i < j ? i : j;
            int64_t o = ptr[e];
            for (int f = b0; f < b1; ++f) {
                const int k = colidx[f];
                if (k >= lim) break;
                const int g = find_upper(rowptr, colidx, diag_pos, k, j);
                if (g >= 0) {
                    const int v2 = lb + (f - b0);
                    const int v3 = ZL + n + urow[k] + (g - diag_pos[k] - 1);
                    if (staged) {
                        const int t = (int)(o - pbase);
                        sh[0][t] = f;
                        sh[1][t] = g;
                        sh[2][t] = v2;
                        sh[3][t] = v3;
                    } else {
                        pik[o] = f;
                        pkj[o] = g;
                        sik[o] = v2;
                        skj[o] = v3;
                    }
                    ++o;
                }
            }
        }
    }
    __syncthreads();
    if (staged) {
        for (int t = threadIdx.x; t < (int)plen; t += blockDim.x) {
            pik[pbase + t] = sh[0][t];
            pkj[pbase + t] = sh[1][t];
            sik[pbase + t] = sh[2][t];
            skj[pbase + t] = sh[3][t];
        }
    }
}

// structural symmetry: one thread per block row; sets *asym when some (i,j) in S_B has no (j,i)
__device__ __forceinline__ void pat_sym_body(int blk, int n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ colidx, unsigned *__restrict__ asym) {
    int i = blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int j = colidx[e];
        if (j != i && find_col(rowptr, colidx, j, i) < 0) {
            atomicOr(asym, 1u);
            return;
        }
    }
}

// per-row counts of strictly lower / upper blocks
__device__ __forceinline__ void pat_tri_counts_body(int blk, int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ diag_pos,
                                 int64_t *__restrict__ nl, int64_t *__restrict__ nu) {
    int i = blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    nl[i] = diag_pos[i] - rowptr[i];
    nu[i] = rowptr[i + 1] - diag_pos[i] - 1;
}

// columns of the lower and upper parts in factor-layout order
__device__ __forceinline__ void pat_tri_cols_body(int blk, int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                               const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow,
                               const int32_t *__restrict__ urow, int32_t *__restrict__ lcol,
                               int32_t *__restrict__ ucol) {
    int i = blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b0 = rowptr[i], d = diag_pos[i], b1 = rowptr[i + 1];
    for (int e = b0; e < d; ++e) lcol[lrow[i] + (e - b0)] = colidx[e];
    for (int e = d + 1; e < b1; ++e) ucol[urow[i] + (e - d - 1)] = colidx[e];
}


// ------------------------------------------------------------------ request generator
constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr uint64_t STREAM_MUL = 0xD1B54A32D192ED03ull;
enum { S_FACE_W = 1, S_OFFDIAG = 2, S_DIAGPERT = 3, S_RHS = 4, S_SPLIT = 5 };

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}
__device__ inline uint64_t key(uint64_t seed, uint64_t stream) { return mix64(seed * GOLDEN + stream * STREAM_MUL); }
__device__ inline double u01(uint64_t k, uint64_t idx) {
    return (double)(mix64(k + idx * GOLDEN) >> 11) * (1.0 / 9007199254740992.0);
}
// lo + (hi - lo) u without a fused multiply-add, like the host generator
__device__ inline double uab(uint64_t k, uint64_t idx, double lo, double hi) {
    return __dadd_rn(lo, __dmul_rn(hi - lo, u01(k, idx)));
}

// Neighbours of a cell in four fixed slots (absent ones have col = -1), as separate scalar
// arrays indexed by compile-time constants so that they stay in registers.
struct Nbs {
    int col[4];       // neighbour cell (output numbering), -1: none
    int64_t face[4];  // natural face index
    int dir[4];       // 0: this cell is the face's first cell (counter 2f), 1: second (2f + 1)
    double scale[4];  // face weight factor (anisotropy)
};

__device__ __forceinline__ void set_nb(Nbs &b, int q, int col, int64_t face, int dir, double scale) {
    b.col[q] = col;
    b.face[q] = face;
    b.dir[q] = dir;
    b.scale[q] = scale;
}

__device__ __forceinline__ bool tri_diag(uint64_t ksplit, int q) { return u01(ksplit, (uint64_t)q) < 0.5; }  // '\'

template <int KIND>
__device__ __forceinline__ void neighbours(int nx, int ny, uint64_t ksplit, int c, int *nat, Nbs &b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) set_nb(b, q, -1, 0, 0, 1.0);
    if constexpr (KIND == ABILU_GEN_TRI) {
        // natural order: cell 2q + t, quad q = iy*nx + ix
        const int q = c >> 1, t = c & 1, ix = q % nx, iy = q / nx;
        const int64_t nq = (int64_t)nx * ny;
        const bool dq = tri_diag(ksplit, q);
        *nat = c;
        // diagonal face q: first cell 2q, second 2q+1
        set_nb(b, 0, t == 0 ? 2 * q + 1 : 2 * q, (int64_t)q, t, 1.0);
        const int64_t hface_l = nq + (int64_t)iy * (nx - 1) + (ix - 1);   // left edge of the quad
        const int64_t hface_r = nq + (int64_t)iy * (nx - 1) + ix;         // right edge
        // the triangle on the left edge of quad q (second cell of that face) or on its right edge
        // (first cell); the neighbour across is the right / left owner of the adjacent quad.
        // Each slot is written once, from selected values.
        const bool on_left = (t == 0) == dq;
        if (on_left ? ix > 0 : ix < nx - 1) {
            const int qq = on_left ? q - 1 : q + 1;
            const bool dd = tri_diag(ksplit, qq);
            const int col = (on_left == dd) ? 2 * qq + 1 : 2 * qq;
            set_nb(b, 2, col, on_left ? hface_l : hface_r, on_left ? 1 : 0, 1.0);
        }
        // bottom edge (t = 0, second cell of the face below) or top edge (t = 1, first cell)
        if (t == 0 ? iy > 0 : iy < ny - 1) {
            const int row = t == 0 ? iy - 1 : iy;
            set_nb(b, 1, t == 0 ? 2 * (q - nx) + 1 : 2 * (q + nx), nq + (int64_t)ny * (nx - 1) + (int64_t)row * nx + ix,
                   t == 0 ? 1 : 0, 1.0);
        }
    } else {
        // line order: output c = t*ny + k (t along the wall, k wall-normal); natural k*nx + t
        const int t = c / ny, k = c % ny;
        *nat = k * nx + t;
        const int64_t nh = (int64_t)ny * (nx - 1);
        const double e = ny > 1 ? 1.0 / (double)(ny - 1) : 0.0;
        if (t > 0) set_nb(b, 0, (t - 1) * ny + k, (int64_t)k * (nx - 1) + (t - 1), 1, 1.0);
        if (t < nx - 1) set_nb(b, 1, (t + 1) * ny + k, (int64_t)k * (nx - 1) + t, 0, 1.0);
        if (k > 0) {
            const double a0 = pow(1000.0, 1.0 - (double)(k - 1) * e), a1 = pow(1000.0, 1.0 - (double)k * e);
            set_nb(b, 2, c - 1, nh + (int64_t)(k - 1) * nx + t, 1, sqrt(a0 * a1));
        }
        if (k < ny - 1) {
            const double a0 = pow(1000.0, 1.0 - (double)k * e), a1 = pow(1000.0, 1.0 - (double)(k + 1) * e);
            set_nb(b, 3, c + 1, nh + (int64_t)k * nx + t, 0, sqrt(a0 * a1));
        }
    }
}

__device__ __forceinline__ void cswap(Nbs &b, int i, int j) {
    const int ki = b.col[i] < 0 ? INT_MAX : b.col[i], kj = b.col[j] < 0 ? INT_MAX : b.col[j];
    const bool sw = kj < ki;
    const int c0 = b.col[i], d0 = b.dir[i];
    const int64_t f0 = b.face[i];
    const double s0 = b.scale[i];
    b.col[i] = sw ? b.col[j] : c0;
    b.face[i] = sw ? b.face[j] : f0;
    b.dir[i] = sw ? b.dir[j] : d0;
    b.scale[i] = sw ? b.scale[j] : s0;
    b.col[j] = sw ? c0 : b.col[j];
    b.face[j] = sw ? f0 : b.face[j];
    b.dir[j] = sw ? d0 : b.dir[j];
    b.scale[j] = sw ? s0 : b.scale[j];
}

template <int KIND>
__device__ __forceinline__ void gen_rowlen_body(int blk, int nx, int ny, uint64_t seed, int n, int64_t *len) {
    const int c = blk * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Nbs b;
    int nat;
    neighbours<KIND>(nx, ny, key(seed, S_SPLIT), c, &nat, b);
    int m = 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) m += b.col[q] >= 0;
    len[c] = m;
}

// One quad per row; lane r writes row r of every block of the row.
template <int KIND>
__device__ __forceinline__ void gen_fill_body(int blk, int nx, int ny, double cfl, uint64_t seed, int n,
                                                 const int32_t *__restrict__ rowptr, int32_t *__restrict__ colidx,
                                                 double *__restrict__ A, double *__restrict__ b) {
    const int c = blk * ROWS_PER_WG + (threadIdx.x >> 2);
    const int r = threadIdx.x & 3;
    if (c >= n) return;
    Nbs nb;
    int nat;
    neighbours<KIND>(nx, ny, key(seed, S_SPLIT), c, &nat, nb);
    // sorting network on the four slots (absent slots last)
    cswap(nb, 0, 1);
    cswap(nb, 2, 3);
    cswap(nb, 0, 2);
    cswap(nb, 1, 3);
    cswap(nb, 1, 2);
    const uint64_t kw = key(seed, S_FACE_W), ko = key(seed, S_OFFDIAG), kp = key(seed, S_DIAGPERT),
                   kr = key(seed, S_RHS);
    int pos = rowptr[c];
    double nrm = 0.0;
    int diag_slot = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (nb.col[q] < 0) continue;
        if (diag_slot < 0 && nb.col[q] > c) {   // the diagonal goes before the first larger column
            diag_slot = pos++;
            if (r == 0) colidx[diag_slot] = c;
        }
        const double w = __dmul_rn(uab(kw, (uint64_t)nb.face[q], 0.5, 1.5), nb.scale[q]);
        const uint64_t ctr = 2 * (uint64_t)nb.face[q] + (uint64_t)nb.dir[q];
        double v[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) v[cc] = __dmul_rn(uab(ko, ctr * 16 + (uint64_t)(r * 4 + cc), -1.0, 1.0), w);
        double *dst = A + (int64_t)pos * BB + r * 4;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) dst[cc] = v[cc];
        if (r == 0) colidx[pos] = nb.col[q];
        // induced 1-norm: max over columns of the absolute column sums (rows are spread over the quad)
        double cs[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            double x[4];
            gather_vec(fabs(v[cc]), x);
            cs[cc] = ((x[0] + x[1]) + x[2]) + x[3];
        }
        nrm += fmax(fmax(cs[0], cs[1]), fmax(cs[2], cs[3]));
        ++pos;
    }
    if (diag_slot < 0) {
        diag_slot = pos;
        if (r == 0) colidx[diag_slot] = c;
    }
    const double shift = nrm / cfl;
    double *dst = A + (int64_t)diag_slot * BB + r * 4;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        double p = uab(kp, (uint64_t)nat * 16 + (uint64_t)(r * 4 + cc), -0.1, 0.1);
        dst[cc] = (cc == r) ? __dadd_rn(p, __dadd_rn(shift, nrm)) : p;
    }
    b[(int64_t)c * 4 + r] = uab(kr, (uint64_t)nat * 4 + r, -1.0, 1.0);
}


}  // namespace abilu_setup
