// Device bodies of the library's kernels, shared by the single-request kernels (one system per
// launch) and the batched serving kernels (one launch over the tiles of many systems). Every body
// takes its tile index `blk` explicitly; the arithmetic lives only here.
#pragma once

#include <type_traits>

#include "abilu_internal.h"

namespace abilu_k {

using namespace abilu;
using namespace abilu_dev;

constexpr int CH = 2;                        // factor sweep: blocks of a row loaded together
// Waves per SIMD the single-precision factor sweeps are compiled for (at most 102 VGPRs). The
// first sweep from A, which inverts a gathered A_jj for each of the two lower blocks in flight,
// would otherwise take 107 VGPRs and run 4 waves; it fits 5 without spilling. The FP64 sweeps
// keep the compiler's choice (at this budget they would spill).
template <typename T>
constexpr int sweep_waves() { return sizeof(T) == 4 ? 5 : 1; }
// apply sweeps: block rows per quad (FP32: two rows keep enough loads in flight; FP64 rows carry
// twice the bytes and run faster one per quad) and rows per workgroup
template <typename T>
constexpr int rpq() { return sizeof(T) == 8 ? 1 : 2; }
template <typename T>
constexpr int rows_per_wg2() { return rpq<T>() * ROWS_PER_WG; }
constexpr int MAX_RESTART = 256;
constexpr int SPMV_ROWS = WG / 8;            // SpMV: eight lanes per block row

// status slots (double[8] in the workspace header, copied to the host)
enum { ST_EST = 0, ST_HN = 1, ST_BETA = 2, ST_NUM = 3, ST_GUARD = 4 };
// misc slots (double[16])
enum { MI_NRM0 = 0, MI_NRM1 = 1, MI_HN = 2, MI_BETA = 3, MI_DONE = 14, MI_GUARD = 15 };

template <typename T, typename S>
__device__ __forceinline__ void load_block_row(const S *base, int64_t pos, int r, T (&v)[4]) {
    load_row(base + pos * BB, r, v);
}

// t -= sum over the update set [p0, p1) of X_ik X_kj (this lane's row of the products).
// L_ik from XL at factor-layout positions (or from A at CSR positions when L_FROM_A),
// X_kj from XU likewise (or A when U_FROM_A).
template <typename T, bool L_FROM_A, bool U_FROM_A>
__device__ __forceinline__ void update_terms(int p0, int p1, int r, const int32_t *__restrict__ pik,
                                             const int32_t *__restrict__ pkj, const int32_t *__restrict__ sik,
                                             const int32_t *__restrict__ skj, const double *__restrict__ A,
                                             const T *XL, const T *XU, T (&t)[4]) {
    for (int q = p0; q < p1; ++q) {
        T l[4], u[4];
        if constexpr (L_FROM_A) load_block_row(A, pik[q], r, l);
        else load_block_row(XL, sik[q], r, l);
        if constexpr (U_FROM_A) load_block_row(A, pkj[q], r, u);
        else load_block_row(XU, skj[q], r, u);
        row_times_block_sub(l, u, t);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ bool skipped(const int *guard) { return guard && *guard == 0; }

// Forward sweep on rows ib, ib + stride, ... (rpq<T>() rows per quad; rows >= n are skipped).
template <typename T, typename YI, bool EMIT_Z>
__device__ __forceinline__ void fwd_rows(int ib, int stride, int n, const int32_t *__restrict__ lrow,
                                         const int32_t *__restrict__ lcol, const T *__restrict__ Lb,
                                         const double *__restrict__ rhs, const YI *yin, T *yout,
                                         const T *__restrict__ Dinv, T *__restrict__ zout) {
    constexpr int RPQ = rpq<T>();
    const int r = threadIdx.x & 3;
    if (ib >= n) return;
    int ii[RPQ], b0[RPQ], b1[RPQ];
    T acc[RPQ];
#pragma unroll
    for (int h = 0; h < RPQ; ++h) {
        ii[h] = ib + h * stride;
        const int i = min(ii[h], n - 1);
        b0[h] = lrow[i];
        b1[h] = (ii[h] < n) ? lrow[i + 1] : b0[h];
        acc[h] = (T)rhs[(int64_t)i * 4 + r];
    }
    int cnt = 0;
#pragma unroll
    for (int h = 0; h < RPQ; ++h) cnt = max(cnt, b1[h] - b0[h]);
    for (int t0 = 0; t0 < cnt; t0 += 2) {
        int j[RPQ][2];
        T l[RPQ][2][4], yv[RPQ][2];
#pragma unroll
        for (int h = 0; h < RPQ; ++h)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = (b1[h] > b0[h]) ? min(b0[h] + t0 + u, b1[h] - 1) : 0;
                j[h][u] = lcol[e];
                load_row(Lb + (int64_t)e * BB, r, l[h][u]);
            }
#pragma unroll
        for (int h = 0; h < RPQ; ++h)
#pragma unroll
            for (int u = 0; u < 2; ++u) yv[h][u] = (T)yin[(int64_t)j[h][u] * 4 + r];
#pragma unroll
        for (int h = 0; h < RPQ; ++h)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                T yj[4];
                gather_vec(yv[h][u], yj);
                const T c = dot4(l[h][u][0], yj[0], l[h][u][1], yj[1], l[h][u][2], yj[2], l[h][u][3], yj[3]);
                acc[h] -= (b0[h] + t0 + u < b1[h]) ? c : T(0);
            }
    }
#pragma unroll
    for (int h = 0; h < RPQ; ++h) {
        if (ii[h] < n) {
            yout[(int64_t)ii[h] * 4 + r] = acc[h];
            if constexpr (EMIT_Z) {
                T dr[4], yi[4];
                load_row(Dinv + (int64_t)ii[h] * BB, r, dr);
                gather_vec(acc[h], yi);
                zout[(int64_t)ii[h] * 4 + r] = dot4(dr[0], yi[0], dr[1], yi[1], dr[2], yi[2], dr[3], yi[3]);
            }
        }
    }
}

template <typename T, typename YI, bool EMIT_Z>
__device__ __forceinline__ void fwd_body(int blk, int n, const int32_t *__restrict__ lrow, const int32_t *__restrict__ lcol,
                                            const T *__restrict__ Lb, const double *__restrict__ rhs, const YI *yin,
                                            T *yout, const T *__restrict__ Dinv, T *__restrict__ zout) {
    fwd_rows<T, YI, EMIT_Z>(blk * rows_per_wg2<T>() + (threadIdx.x >> 2), ROWS_PER_WG, n, lrow, lcol, Lb, rhs, yin, yout,
                            Dinv, zout);
}

// Backward sweep on rows ib, ib + stride, ... (rpq<T>() rows per quad).
template <typename T, typename YI, typename ZO, bool OFFDIAG, bool DUAL>
__device__ __forceinline__ void bwd_rows(int ib, int stride, int n, const int32_t *__restrict__ urow,
                                         const int32_t *__restrict__ ucol, const T *__restrict__ Ub,
                                         const T *__restrict__ Dinv, const YI *__restrict__ y, const T *zin, ZO *zout,
                                         T *zout2) {
    constexpr int RPQ = rpq<T>();
    const int r = threadIdx.x & 3;
    if (ib >= n) return;
    int ii[RPQ], b0[RPQ], b1[RPQ];
    T acc[RPQ];
#pragma unroll
    for (int h = 0; h < RPQ; ++h) {
        ii[h] = ib + h * stride;
        const int i = min(ii[h], n - 1);
        acc[h] = (T)y[(int64_t)i * 4 + r];
        if constexpr (OFFDIAG) {
            b0[h] = urow[i];
            b1[h] = (ii[h] < n) ? urow[i + 1] : b0[h];
        }
    }
    if constexpr (OFFDIAG) {
        int cnt = 0;
#pragma unroll
        for (int h = 0; h < RPQ; ++h) cnt = max(cnt, b1[h] - b0[h]);
        for (int t0 = 0; t0 < cnt; t0 += 2) {
            int j[RPQ][2];
            T u4[RPQ][2][4], zv[RPQ][2];
#pragma unroll
            for (int h = 0; h < RPQ; ++h)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = (b1[h] > b0[h]) ? min(b0[h] + t0 + u, b1[h] - 1) : 0;
                    j[h][u] = ucol[e];
                    load_row(Ub + (int64_t)e * BB, r, u4[h][u]);
                }
#pragma unroll
            for (int h = 0; h < RPQ; ++h)
#pragma unroll
                for (int u = 0; u < 2; ++u) zv[h][u] = zin[(int64_t)j[h][u] * 4 + r];
#pragma unroll
            for (int h = 0; h < RPQ; ++h)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    T zj[4];
                    gather_vec(zv[h][u], zj);
                    const T c = dot4(u4[h][u][0], zj[0], u4[h][u][1], zj[1], u4[h][u][2], zj[2], u4[h][u][3], zj[3]);
                    acc[h] -= (b0[h] + t0 + u < b1[h]) ? c : T(0);
                }
        }
    }
#pragma unroll
    for (int h = 0; h < RPQ; ++h) {
        if (ii[h] < n) {
            T dr[4], a[4];
            load_row(Dinv + (int64_t)ii[h] * BB, r, dr);
            gather_vec(acc[h], a);
            const T z = dot4(dr[0], a[0], dr[1], a[1], dr[2], a[2], dr[3], a[3]);
            zout[(int64_t)ii[h] * 4 + r] = (ZO)z;
            if constexpr (DUAL) zout2[(int64_t)ii[h] * 4 + r] = z;
        }
    }
}

template <typename T, typename YI, typename ZO, bool OFFDIAG, bool DUAL>
__device__ __forceinline__ void bwd_body(int blk, int n, const int32_t *__restrict__ urow, const int32_t *__restrict__ ucol,
                                            const T *__restrict__ Ub, const T *__restrict__ Dinv,
                                            const YI *__restrict__ y, const T *zin, ZO *zout, T *zout2) {
    bwd_rows<T, YI, ZO, OFFDIAG, DUAL>(blk * rows_per_wg2<T>() + (threadIdx.x >> 2), ROWS_PER_WG, n, urow, ucol, Ub, Dinv, y,
                                       zin, zout, zout2);
}

template <bool RESID>
__device__ __forceinline__ void spmv_body(int blk, int n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ colidx, const double *__restrict__ A,
                                             const double *__restrict__ x, double *__restrict__ y,
                                             const double *__restrict__ b) {
    // eight lanes per block row (SPMV_ROWS rows per workgroup): lane l takes row l / 2, columns
    // 2 (l % 2) and 2 (l % 2) + 1 of every block, so each load instruction covers whole 128-byte
    // FP64 blocks (a quad per row covers half of each block per instruction and reads each line
    // in two passes: 4-5% slower on the 4M-cell matrix)
    constexpr int SCH = 4;
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int i = blk * SPMV_ROWS + (threadIdx.x >> 3);
    const int rr = (threadIdx.x >> 1) & 3, h = threadIdx.x & 1;
    if (i >= n) return;
    const int b0 = rowptr[i], b1 = rowptr[i + 1];
    double acc = 0.0;
    for (int e0 = b0; e0 < b1; e0 += SCH) {
        int j[SCH];
        d2 a[SCH], xv[SCH];
#pragma unroll
        for (int u = 0; u < SCH; ++u) {
            const int e = min(e0 + u, b1 - 1);
            j[u] = colidx[e];
            a[u] = *reinterpret_cast<const d2 *>(A + (int64_t)e * BB + rr * 4 + 2 * h);
        }
#pragma unroll
        for (int u = 0; u < SCH; ++u) xv[u] = *reinterpret_cast<const d2 *>(x + (int64_t)j[u] * 4 + 2 * h);
#pragma unroll
        for (int u = 0; u < SCH; ++u) {
            const double c = a[u].x * xv[u].x + a[u].y * xv[u].y;
            acc += (e0 + u < b1) ? c : 0.0;
        }
    }
    acc += __shfl_xor(acc, 1, 64);   // the row's other two columns, from the neighbouring lane
    if (h == 0) y[(int64_t)i * 4 + rr] = RESID ? b[(int64_t)i * 4 + rr] - acc : acc;
}

__device__ __forceinline__ void mdot_body(int blk, int64_t len, const double *__restrict__ V, int64_t ldv, int q,
                                             const double *__restrict__ w, double *__restrict__ partial, int nb,
                                             const int *guard) {
    if (skipped(guard)) return;
    __shared__ double sh[MAX_RESTART + 2][WG / 64];
    const int64_t base = (int64_t)blk * VEC_TILE + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double wv[VEC_E];
    const bool full = base + (int64_t)(VEC_E - 1) * WG < len;
#pragma unroll
    for (int e = 0; e < VEC_E; ++e) {
        const int64_t t = base + (int64_t)e * WG;
        wv[e] = (full || t < len) ? w[t] : 0.0;
    }
    for (int k = 0; k < q; ++k) {
        const double *vk = V + (int64_t)k * ldv;
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < VEC_E; ++e) {
            const int64_t t = base + (int64_t)e * WG;
            s += ((full || t < len) ? vk[t] : 0.0) * wv[e];
        }
        s = wave_sum(s);
        if (lane == 0) sh[k][wave] = s;
    }
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < VEC_E; ++e) s += wv[e] * wv[e];
    s = wave_sum(s);
    if (lane == 0) sh[q][wave] = s;
    __syncthreads();
    for (int k = threadIdx.x; k <= q; k += WG)
        partial[(int64_t)k * nb + blk] = ((sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]));
}

__device__ __forceinline__ void update_body(int blk, int64_t len, const double *__restrict__ V, int64_t ldv, int q,
                                               const double *__restrict__ c, double alpha, double *__restrict__ w,
                                               double *__restrict__ partial, const int *guard) {
    if (skipped(guard)) return;
    __shared__ double sh[WG / 64];
    const int64_t base = (int64_t)blk * VEC_TILE + threadIdx.x;
    const bool full = base + (int64_t)(VEC_E - 1) * WG < len;
    double acc[VEC_E];
#pragma unroll
    for (int e = 0; e < VEC_E; ++e) {
        const int64_t t = base + (int64_t)e * WG;
        acc[e] = (full || t < len) ? w[t] : 0.0;
    }
    for (int k = 0; k < q; ++k) {
        const double ck = alpha * c[k];
        const double *vk = V + (int64_t)k * ldv;
#pragma unroll
        for (int e = 0; e < VEC_E; ++e) {
            const int64_t t = base + (int64_t)e * WG;
            acc[e] += ck * ((full || t < len) ? vk[t] : 0.0);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < VEC_E; ++e) {
        const int64_t t = base + (int64_t)e * WG;
        if (full || t < len) w[t] = acc[e];
        s += acc[e] * acc[e];
    }
    if (partial) {
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) partial[blk] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    }
}

__device__ __forceinline__ void reduce_cols_body(int blk, const double *__restrict__ partial, int nb,
                                                    double *__restrict__ out, const int *guard) {
    if (skipped(guard)) return;
    __shared__ double sh[WG / 64];
    const double *pc = partial + (int64_t)blk * nb;
    // eight independent partial sums keep eight loads in flight per lane (fixed order: entry b
    // goes to sum (b / WG) mod 8 while whole groups of 8 WG entries remain, the rest to sum 0)
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0, a6 = 0.0, a7 = 0.0;
    int b = threadIdx.x;
    for (; b + 7 * WG < nb; b += 8 * WG) {
        a0 += pc[b];
        a1 += pc[b + WG];
        a2 += pc[b + 2 * WG];
        a3 += pc[b + 3 * WG];
        a4 += pc[b + 4 * WG];
        a5 += pc[b + 5 * WG];
        a6 += pc[b + 6 * WG];
        a7 += pc[b + 7 * WG];
    }
    for (; b < nb; b += WG) a0 += pc[b];
    double s = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blk] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__device__ __forceinline__ void scale_body(int blk, int64_t len, const double *w, double *v, const double *h) {
    const double hv = *h;
    const int64_t base = (int64_t)blk * VEC_TILE + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_E; ++e) {
        const int64_t t = base + (int64_t)e * WG;
        if (t < len) v[t] = (hv != 0.0) ? w[t] / hv : w[t];
    }
}

__device__ __forceinline__ void gs1_body(int blk, int k, int m, const double *__restrict__ red, double *H, double *coef, double *misc) {
    for (int q = 0; q <= k; ++q) {
        H[(int64_t)k * (m + 1) + q] = red[q];
        coef[q] = red[q];
    }
    misc[MI_NRM0] = sqrt(red[k + 1]);
}

__device__ __forceinline__ void gs1_done_body(int blk, const double *__restrict__ nrm2, double *misc, int *guard) {
    const double n1 = sqrt(nrm2[0]);
    misc[MI_NRM1] = n1;
    *guard = (n1 < 0.70710678118654752440 * misc[MI_NRM0]) ? 1 : 0;
}

__device__ __forceinline__ void gs2_body(int blk, int k, int m, const double *__restrict__ red, double *H, double *coef, const int *guard) {
    if (*guard == 0) return;
    for (int q = 0; q <= k; ++q) {
        H[(int64_t)k * (m + 1) + q] += red[q];
        coef[q] = red[q];
    }
}

__device__ __forceinline__ void givens_body(int blk, int k, int m, const double *__restrict__ nrm2_pass2, const int *guard, double *H,
                         double *cs, double *sn, double *g, double *misc, double *status) {
    const double hn = (*guard) ? sqrt(nrm2_pass2[0]) : misc[MI_NRM1];
    double *h = H + (int64_t)k * (m + 1);
    h[k + 1] = hn;
    for (int q = 0; q < k; ++q) {
        const double a = h[q], b = h[q + 1];
        h[q] = cs[q] * a + sn[q] * b;
        h[q + 1] = -sn[q] * a + cs[q] * b;
    }
    const double a = h[k], b = h[k + 1];
    const double rho = sqrt(a * a + b * b);
    cs[k] = rho > 0 ? a / rho : 1.0;
    sn[k] = rho > 0 ? b / rho : 0.0;
    h[k] = rho;
    h[k + 1] = 0.0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    misc[MI_HN] = hn;
    status[ST_EST] = fabs(g[k + 1]);
    status[ST_HN] = hn;
    status[ST_GUARD] = (double)(*guard);
}

__device__ __forceinline__ void solve_body(int blk, int k, int m, const double *__restrict__ H, const double *__restrict__ g, double *coef) {
    for (int q = k - 1; q >= 0; --q) {
        double s = g[q];
        for (int t = q + 1; t < k; ++t) s -= H[(int64_t)t * (m + 1) + q] * coef[t];
        coef[q] = s / H[(int64_t)q * (m + 1) + q];
    }
}

__device__ __forceinline__ void beta_body(int blk, int m, const double *__restrict__ red, double *g, double *misc, double *status, int slot) {
    const double beta = sqrt(red[0]);
    status[slot] = beta;
    misc[MI_BETA] = beta;
    if (g) {
        g[0] = beta;
        for (int q = 1; q <= m + 1; ++q) g[q] = 0.0;
    }
}

__device__ __forceinline__ void zero_body(int blk, int64_t len, double *v) {
    const int64_t base = (int64_t)blk * VEC_TILE + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_E; ++e) {
        const int64_t t = base + (int64_t)e * WG;
        if (t < len) v[t] = 0.0;
    }
}

template <typename T, typename S, bool SRC_CSR, bool COPY>
__device__ __forceinline__ void factor_init_body(int blk, int n, int ZL, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ diag_pos,
                                                    const int32_t *__restrict__ lrow,
                                                    const int32_t *__restrict__ urow, const S *X0, T *Xout, T *D0,
                                                    unsigned *flags) {
    const int i = blk * ROWS_PER_WG + (threadIdx.x >> 2);
    const int r = threadIdx.x & 3;
    if (i >= n) return;
    if constexpr (COPY) {
        static_assert(SRC_CSR, "copy reads A");
        const int b0 = rowptr[i], d = diag_pos[i], b1 = rowptr[i + 1];
        const int lb = lrow[i], ub = urow[i];
        for (int e = b0; e < b1; ++e) {
            T v[4];
            load_row(X0 + (int64_t)e * BB, r, v);
            store_row(Xout + (int64_t)split_pos(e, i, b0, d, lb, ub, ZL, n) * BB, r, v);
        }
    }
    const int64_t dpos = SRC_CSR ? (int64_t)diag_pos[i] : (int64_t)ZL + i;
    T u[4], M[16], out[4];
    load_row(X0 + dpos * BB, r, u);
    gather_block(u, M);
    bool ok = inv4_row(M, r, out);
    store_row(D0 + (int64_t)i * BB, r, out);
    if (!ok && r == 0) atomicOr(flags, ABILU_FLAG_MODIFIED);
}

// One sweep over block row i (a quad of 4 lanes). The strictly lower blocks are loaded in chunks
// of CHL (their A blocks and inverses fetched together) and computed and stored one at a time in
// ascending column order, so a block whose update set holds an earlier block of the row reads that
// block's value from this sweep when the sweep works in place (the strict Gauss-Seidel order within
// the row). This also keeps the first in-place sweep from A from reading the output buffer before
// this sweep has written it: there X_ik of the row is never taken from the initial guess.
// D_FROM_A (first sweep from the initial guess X0 = A): the inverses U_jj^{-1} = A_jj^{-1} the
// lower blocks need are formed here from A, in the same arithmetic as the initialisation kernel,
// so no separate pass writes and re-reads them. A row whose A_ii no other row inverts this way
// inverts it once itself, only to raise the flag the initialisation would raise when that inverse
// is replaced: with sym (structurally symmetric pattern) those are the rows without strictly upper
// blocks, otherwise every row checks its own.
template <typename T, bool L_FROM_A, bool U_FROM_A, int CHL = CH, bool D_FROM_A = false>
__device__ __forceinline__ void factor_sweep_row(int i,
    int n, int ZL, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
    const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ pik, const int32_t *__restrict__ pkj,
    const int32_t *__restrict__ sik, const int32_t *__restrict__ skj, const double *__restrict__ A, const T *XL,
    const T *XU, const T *Dp, T *Xn, T *Dn, unsigned *flags, bool sym = false) {
    const int r = threadIdx.x & 3;
    if (i >= n) return;
    const int b0 = rowptr[i], b1 = rowptr[i + 1], d = diag_pos[i];
    const int lbase = lrow[i], ubase = urow[i];
    // update-set extents: lower blocks [pb0, pd), diagonal [pd, pd1), upper [pd1, pb1)
    const int pb0 = pair_ptr[b0], pd = pair_ptr[d], pd1 = pair_ptr[d + 1], pb1 = pair_ptr[b1];
    T *XnL = Xn + (int64_t)lbase * BB;
    T *XnU = Xn + ((int64_t)ZL + n + ubase) * BB;
    unsigned fl = 0;

    // strictly lower blocks: L_ij = (A_ij - sum) U_jj^{-1}
    for (int e0 = b0; e0 < d; e0 += CHL) {
        T t[CHL][4], dr[CHL][4];
        int j[CHL];
#pragma unroll
        for (int u = 0; u < CHL; ++u) {
            const int e = min(e0 + u, d - 1);
            load_row(A + (int64_t)e * BB, r, t[u]);
            j[u] = colidx[e];
        }
        if constexpr (D_FROM_A) {
#pragma unroll
            for (int u = 0; u < CHL; ++u) {
                T a[4], M[16];
                load_row(A + (int64_t)diag_pos[j[u]] * BB, r, a);
                gather_block(a, M);
                if (!inv4_row(M, r, dr[u])) fl |= ABILU_FLAG_MODIFIED;
            }
        } else {
#pragma unroll
            for (int u = 0; u < CHL; ++u) load_row(Dp + (int64_t)j[u] * BB, r, dr[u]);
        }
#pragma unroll
        for (int u = 0; u < CHL; ++u) {
            if (e0 + u < d) {
                if (pd > pb0)
                    update_terms<T, L_FROM_A, U_FROM_A>(pair_ptr[e0 + u], pair_ptr[e0 + u + 1], r, pik, pkj, sik,
                                                        skj, A, XL, XU, t[u]);
                T x[4];
                row_times_block(t[u], dr[u], x);
                fl |= nonfinite4(x);
                store_row(XnL + (int64_t)(e0 + u - b0) * BB, r, x);
            }
        }
    }
    // diagonal block U_ii = A_ii - sum, and its inverse
    {
        T t[4];
        load_row(A + (int64_t)d * BB, r, t);
        if constexpr (D_FROM_A) {
            if (!sym || d + 1 == b1) {
                T M[16], unused[4];
                gather_block(t, M);
                if (!inv4_row(M, r, unused)) fl |= ABILU_FLAG_MODIFIED;
            }
        }
        update_terms<T, L_FROM_A, U_FROM_A>(pd, pd1, r, pik, pkj, sik, skj, A, XL, XU, t);
        fl |= nonfinite4(t);
        store_row(Xn + ((int64_t)ZL + i) * BB, r, t);
        T M[16], out[4];
        gather_block(t, M);
        if (!inv4_row(M, r, out)) fl |= ABILU_FLAG_MODIFIED;
        store_row(Dn + (int64_t)i * BB, r, out);
    }
    // strictly upper blocks: U_ij = A_ij - sum
    for (int e0 = d + 1; e0 < b1; e0 += CH) {
        T t[CH][4];
#pragma unroll
        for (int u = 0; u < CH; ++u) load_row(A + (int64_t)min(e0 + u, b1 - 1) * BB, r, t[u]);
        if (pb1 > pd1) {
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (e0 + u < b1)
                    update_terms<T, L_FROM_A, U_FROM_A>(pair_ptr[e0 + u], pair_ptr[e0 + u + 1], r, pik, pkj, sik,
                                                        skj, A, XL, XU, t[u]);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (e0 + u < b1) {
                fl |= nonfinite4(t[u]);
                store_row(XnU + (int64_t)(e0 + u - d - 1) * BB, r, t[u]);
            }
        }
    }
    if (fl) atomicOr(flags, fl);
}

// t -= sum over the update set [p0, p1) of X_ik X_kj for a row of a chunk (chunked sweeps).
// X_ik is a block of this row and comes from Xn (this sweep). X_kj lies in the strictly upper part
// of row k < i: rows of the chunk (factor-layout position >= ubound) come from Xn, earlier rows
// from XO, or from A at CSR positions when OUT_FROM_A (the first sweep from X0 = A). PAIR2 takes
// the pairs two at a time (clamped index loads, then the four block rows) so that a row's chain of
// dependent loads is short, at the cost of registers; either way the products are subtracted in
// the list's order, so both forms give the same values.
template <typename T, bool OUT_FROM_A>
__device__ __forceinline__ void load_u_chunk(int q, int sp, int ubound, int r, const int32_t *__restrict__ pkj,
                                             const double *__restrict__ A, const T *Xn, const T *XO, T (&u)[4]) {
    if (sp >= ubound) load_block_row(Xn, sp, r, u);
    else if constexpr (OUT_FROM_A) load_block_row(A, pkj[q], r, u);
    else load_block_row(XO, sp, r, u);
}

template <typename T, bool OUT_FROM_A, bool PAIR2>
__device__ __forceinline__ void update_terms_chunk(int p0, int p1, int r, int ubound, const int32_t *__restrict__ pkj,
                                                   const int32_t *__restrict__ sik, const int32_t *__restrict__ skj,
                                                   const double *__restrict__ A, const T *Xn, const T *XO,
                                                   T (&t)[4]) {
    if constexpr (PAIR2) {
        for (int q0 = p0; q0 < p1; q0 += 2) {
            const int qb = min(q0 + 1, p1 - 1);
            const int sa = sik[q0], sb = sik[qb];
            const int ka = skj[q0], kb = skj[qb];
            T la[4], lb[4], ua[4], ub[4];
            load_block_row(Xn, sa, r, la);
            load_block_row(Xn, sb, r, lb);
            load_u_chunk<T, OUT_FROM_A>(q0, ka, ubound, r, pkj, A, Xn, XO, ua);
            load_u_chunk<T, OUT_FROM_A>(qb, kb, ubound, r, pkj, A, Xn, XO, ub);
            row_times_block_sub(la, ua, t);
            if (q0 + 1 < p1) row_times_block_sub(lb, ub, t);
        }
    } else {
        for (int q = p0; q < p1; ++q) {
            T l[4], u[4];
            load_block_row(Xn, sik[q], r, l);
            load_u_chunk<T, OUT_FROM_A>(q, skj[q], ubound, r, pkj, A, Xn, XO, u);
            row_times_block_sub(l, u, t);
        }
    }
}

// One chunked sweep over block row i of the chunk starting at row c0: the blocks of the row in
// ascending column order, each stored before the next is computed (a Gauss-Seidel order within
// the row), reading the chunk's rows from this sweep (Xn, Dn) and earlier rows from XO, DO.
template <typename T, bool OUT_FROM_A, bool PAIR2>
__device__ __forceinline__ void factor_chunk_row(int i, int c0, int ubound,
    int n, int ZL, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
    const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ pkj, const int32_t *__restrict__ sik,
    const int32_t *__restrict__ skj, const double *__restrict__ A, const T *XO, const T *DO, T *Xn, T *Dn,
    unsigned *flags) {
    const int r = threadIdx.x & 3;
    const int b0 = rowptr[i], b1 = rowptr[i + 1], d = diag_pos[i];
    T *XnL = Xn + (int64_t)lrow[i] * BB;
    T *XnU = Xn + ((int64_t)ZL + n + urow[i]) * BB;
    unsigned fl = 0;
    // strictly lower blocks: L_ij = (A_ij - sum) U_jj^{-1}, U_jj^{-1} of this sweep if j is in the
    // chunk. With PAIR2 and no update terms in the row's lower part the blocks are independent and
    // are computed two at a time; otherwise one at a time, each seeing the ones before it.
    if (PAIR2 && pair_ptr[d] == pair_ptr[b0]) {
        for (int e0 = b0; e0 < d; e0 += 2) {
            const int eb = min(e0 + 1, d - 1);
            T ta[4], tb[4], da[4], db[4];
            load_row(A + (int64_t)e0 * BB, r, ta);
            load_row(A + (int64_t)eb * BB, r, tb);
            const int ja = colidx[e0], jb = colidx[eb];
            load_row((ja >= c0 ? (const T *)Dn : DO) + (int64_t)ja * BB, r, da);
            load_row((jb >= c0 ? (const T *)Dn : DO) + (int64_t)jb * BB, r, db);
            T xa[4], xb[4];
            row_times_block(ta, da, xa);
            row_times_block(tb, db, xb);
            fl |= nonfinite4(xa);
            store_row(XnL + (int64_t)(e0 - b0) * BB, r, xa);
            if (e0 + 1 < d) {
                fl |= nonfinite4(xb);
                store_row(XnL + (int64_t)(e0 + 1 - b0) * BB, r, xb);
            }
        }
    } else {
        for (int e = b0; e < d; ++e) {
            T t[4], dr[4];
            load_row(A + (int64_t)e * BB, r, t);
            const int j = colidx[e];
            load_row((j >= c0 ? (const T *)Dn : DO) + (int64_t)j * BB, r, dr);
            update_terms_chunk<T, OUT_FROM_A, PAIR2>(pair_ptr[e], pair_ptr[e + 1], r, ubound, pkj, sik, skj, A, Xn, XO, t);
            T x[4];
            row_times_block(t, dr, x);
            fl |= nonfinite4(x);
            store_row(XnL + (int64_t)(e - b0) * BB, r, x);
        }
    }
    // diagonal block U_ii = A_ii - sum and its inverse
    {
        T t[4];
        load_row(A + (int64_t)d * BB, r, t);
        update_terms_chunk<T, OUT_FROM_A, PAIR2>(pair_ptr[d], pair_ptr[d + 1], r, ubound, pkj, sik, skj, A, Xn, XO, t);
        fl |= nonfinite4(t);
        store_row(Xn + ((int64_t)ZL + i) * BB, r, t);
        T M[16], out[4];
        gather_block(t, M);
        if (!inv4_row(M, r, out)) fl |= ABILU_FLAG_MODIFIED;
        store_row(Dn + (int64_t)i * BB, r, out);
    }
    // strictly upper blocks: U_ij = A_ij - sum (independent of each other)
    for (int e0 = d + 1; e0 < b1; e0 += CH) {
        T t[CH][4];
#pragma unroll
        for (int u = 0; u < CH; ++u) load_row(A + (int64_t)min(e0 + u, b1 - 1) * BB, r, t[u]);
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (e0 + u < b1)
                update_terms_chunk<T, OUT_FROM_A, PAIR2>(pair_ptr[e0 + u], pair_ptr[e0 + u + 1], r, ubound, pkj, sik, skj,
                                                  A, Xn, XO, t[u]);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (e0 + u < b1) {
                fl |= nonfinite4(t[u]);
                store_row(XnU + (int64_t)(e0 + u - d - 1) * BB, r, t[u]);
            }
        }
    }
    if (fl) atomicOr(flags, fl);
}

template <typename T, bool L_FROM_A, bool U_FROM_A, bool D_FROM_A = false>
__device__ __forceinline__ void factor_sweep_body(int blk,
    int n, int ZL, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
    const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ pik, const int32_t *__restrict__ pkj,
    const int32_t *__restrict__ sik, const int32_t *__restrict__ skj, const double *__restrict__ A, const T *XL,
    const T *XU, const T *Dp, T *Xn, T *Dn, unsigned *flags, bool sym = false) {
    factor_sweep_row<T, L_FROM_A, U_FROM_A, CH, D_FROM_A>(blk * ROWS_PER_WG + (threadIdx.x >> 2), n, ZL, rowptr, colidx, diag_pos,
                                            lrow, urow, pair_ptr, pik, pkj, sik, skj, A, XL, XU, Dp, Xn, Dn, flags, sym);
}

// ------------------------------------------------------------------ per-row records of the
// quad-per-chunk runner (layout beside REC_INTS)

// Records are stored as REC_INTS / 4 planes of int4 (plane k holds fields 4k .. 4k + 3 of every
// record), each plane step-major: the record of row c * R + t at index t * nch + c. The quads of a
// wavefront run chunks c, c + 1, ... in lock step, so a load of one plane reads adjacent 16-byte
// pieces, and a sweep that needs only some fields reads only their planes.
__device__ __forceinline__ int4 rec_quad(const int32_t *__restrict__ rec, int R, int c, int nch, int t, int k) {
    return reinterpret_cast<const int4 *>(rec)[(int64_t)k * R * nch + (int64_t)t * nch + c];
}

__device__ __forceinline__ void load_rec(const int32_t *__restrict__ rec, int R, int c, int nch, int t, int4 (&rc)[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) rc[k] = rec_quad(rec, R, c, nch, t, k);
}

template <int K>
__device__ __forceinline__ int rec_field(const int4 (&rc)[6]) {
    if constexpr ((K & 3) == 0) return rc[K >> 2].x;
    else if constexpr ((K & 3) == 1) return rc[K >> 2].y;
    else if constexpr ((K & 3) == 2) return rc[K >> 2].z;
    else return rc[K >> 2].w;
}

// v = rows[k] for a runtime k < N, as a masked blend of the bit patterns: the rows stay in
// registers (a chain of selects between the rows would be folded into a load at a computed offset,
// which forces the rows into scratch memory)
template <typename T, int N>
__device__ __forceinline__ void pick_row(const T (&rows)[N][4], int k, T (&v)[4]) {
    using U = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        U x = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) x |= ((U)0 - (U)(k == q)) & __builtin_bit_cast(U, rows[q][c]);
        v[c] = __builtin_bit_cast(T, x);
    }
}

template <typename T>
__device__ __forceinline__ void copy_row(const T (&a)[4], T (&b)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = a[c];
}

}  // namespace abilu_k
