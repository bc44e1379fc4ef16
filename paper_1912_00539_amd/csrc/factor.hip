// Block ILU(0) factorisation sweeps (Section 4.2).
//
// Every block (i,j) of S_B is an unknown of the fixed-point equations (equation blockH):
//   H_ij(X) = (A_ij - sum_{k in K(i,j)} X_ik X_kj) X_jj^{-1}   for i > j
//   H_ij(X) =  A_ij - sum_{k in K(i,j)} X_ik X_kj              for i <= j
// One sweep evaluates H for every block at once. The diagonal inverses are carried as a second
// array Dinv (the exact 4x4 inversion of each diagonal block, fused into the sweep: the quad that
// produces U_ii inverts it on the spot).
//
// Factor layout: [strictly lower blocks | diagonal blocks | strictly upper blocks], each part in
// row order, so the forward and backward apply sweeps stream one contiguous part each. A stays in
// CSR order. X_ik is always a strictly lower block of row i; X_kj lies in row k < i.
//
// Mapping: one quad of 4 lanes per block row i; lane r owns row r of every 4x4 block of the row
// (a block is one contiguous 64/128-byte access by the quad) and rows of other blocks come from
// the quad by DPP broadcasts. A row's blocks are processed in chunks of CH with branch-free
// (clamped) loads so that several block loads are in flight per lane.
//
// SYNC : reads only X^p, Dinv^p and writes X^{p+1}, Dinv^{p+1} (ping-pong buffers): the
//        Jacobi-type iteration x^{p+1} = h(x^p). Deterministic.
// ASYNC: X and Dinv are updated in place; reads see whatever value is in memory (possibly a block
//        another quad is writing: torn reads are allowed since every scalar has its own delay in
//        the block-asynchronous model). Blocks of a row are updated in ascending column order, so
//        U_ii uses the L_ik this quad has just written. The first sweep from A reads the X_kj of
//        other rows from A itself (the initial guess, the oldest admissible value) and so needs no
//        copy of A into X. Sums are accumulated in registers and stored once; no atomics on values.
// CHUNK_SYNC / CHUNK_ASYNC: a Gauss-Seidel sweep inside each chunk of consecutive rows (rows of
//        other chunks from the previous sweep, or as in memory), run a chunk per workgroup level
//        by level or a chunk per quad row by row. ASYNC_SERIAL: every row in order by one quad.
#include "kernels.h"

using namespace abilu;
using namespace abilu_dev;
using namespace abilu_k;

namespace {

// X0 -> (optional) copy into Xout in factor layout, and D0 = inverses of X0's diagonal blocks.
// SRC_CSR: X0 is A (CSR order, double); otherwise X0 is a factor-layout array of T. Rows are
// independent; the workgroups take them in descending order so that the ascending sweep after it
// starts on the rows whose inverses and diagonal blocks were touched last.
template <typename T, typename S, bool SRC_CSR, bool COPY>
__global__ __launch_bounds__(WG) void k_factor_init(int n, int ZL, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ diag_pos,
                                                    const int32_t *__restrict__ lrow,
                                                    const int32_t *__restrict__ urow, const S *X0, T *Xout, T *D0,
                                                    unsigned *flags) {
    factor_init_body<T, S, SRC_CSR, COPY>(gridDim.x - 1 - blockIdx.x, n, ZL, rowptr, diag_pos, lrow, urow, X0, Xout,
                                          D0, flags);
}

// One sweep (D_FROM_A: the first sweep from A, forming the initial inverses itself; sym: the
// pattern is structurally symmetric).
template <typename T, bool L_FROM_A, bool U_FROM_A, bool D_FROM_A = false>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(sweep_waves<T>()))) void k_factor_sweep(
    int n, int ZL, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
    const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ pik, const int32_t *__restrict__ pkj,
    const int32_t *__restrict__ sik, const int32_t *__restrict__ skj, const double *__restrict__ A, const T *XL,
    const T *XU, const T *Dp, T *Xn, T *Dn, unsigned *flags, int sym) {
    factor_sweep_body<T, L_FROM_A, U_FROM_A, D_FROM_A>(blockIdx.x, n, ZL, rowptr, colidx, diag_pos, lrow, urow, pair_ptr, pik, pkj, sik, skj, A, XL, XU, Dp, Xn, Dn, flags, sym != 0);
}

// The asynchronous sweep with a single worker: one quad over the rows in ascending order, in
// place (a Gauss-Seidel sweep). Launched with one workgroup of 4 lanes.
template <typename T>
__global__ __launch_bounds__(64) void k_factor_sweep_serial(
    int n, int ZL, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
    const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ pik, const int32_t *__restrict__ pkj,
    const int32_t *__restrict__ sik, const int32_t *__restrict__ skj, const double *__restrict__ A, T *X, T *D,
    unsigned *flags) {
    for (int i = 0; i < n; ++i) {
        factor_sweep_row<T, false, false, 1>(i, n, ZL, rowptr, colidx, diag_pos, lrow, urow, pair_ptr, pik, pkj, sik,
                                             skj, A, X, X, D, X, D, flags);
        __threadfence();   // row i's blocks and inverse are visible to the rows after it
    }
}

// One chunked sweep: workgroup c runs chunk c, level by level (lower schedule), one quad per row;
// the barrier after each level makes the level's blocks and inverses visible to the next.
template <typename T, bool OUT_FROM_A>
__global__ __launch_bounds__(WG) void k_factor_sweep_chunk(
    int n, int ZL, int R, const int32_t *__restrict__ order, const int32_t *__restrict__ lvptr,
    const int32_t *__restrict__ lvstart, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
    const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ pkj, const int32_t *__restrict__ sik,
    const int32_t *__restrict__ skj, const double *__restrict__ A, const T *XO, const T *DO, T *Xn, T *Dn,
    unsigned *flags) {
    const int c = blockIdx.x;
    const int c0 = c * R;
    const int ubound = ZL + n + urow[c0];
    const int b = lvptr[c], nl = lvptr[c + 1] - b - 1;
    const int quad = threadIdx.x >> 2;
    for (int l = 0; l < nl; ++l) {
        const int p1 = lvstart[b + l + 1];
        for (int q = lvstart[b + l] + quad; q < p1; q += ROWS_PER_WG)
            factor_chunk_row<T, OUT_FROM_A, false>(order[q], c0, ubound, n, ZL, rowptr, colidx, diag_pos, lrow, urow,
                                                   pair_ptr, pkj, sik, skj, A, XO, DO, Xn, Dn, flags);
        __syncthreads();
    }
}

// One chunked sweep with one quad per chunk running the chunk's rows in ascending order (the
// worker-per-chunk form of the same sweep). Every value of the chunk that a lane reads was stored
// by that same lane (lane r owns row r of every block), so program order makes it visible; the
// values of the row computed just before are taken from registers instead. Each row's operands
// are located by its record (read one row ahead) and fetched together, so a row costs one memory
// round trip. The arithmetic, and its order, is that of factor_chunk_row, which takes the rows a
// record cannot describe.
template <typename T, bool OUT_FROM_A>
__global__ __launch_bounds__(WG) void k_factor_sweep_chunk_rows(
    int n, int ZL, int R, int nch, const int32_t *__restrict__ rec, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ colidx, const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow,
    const int32_t *__restrict__ urow, const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ pkj,
    const int32_t *__restrict__ sik, const int32_t *__restrict__ skj, const double *__restrict__ A, const T *XO,
    const T *DO, T *Xn, T *Dn, unsigned *flags) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    if (c >= nch) return;
    const int r = threadIdx.x & 3;
    const int c0 = c * R, m = min(n, c0 + R) - c0;
    const int ubase = ZL + n;
    const int ubound = ubase + urow[c0];
    T pD[4] = {}, pU[REC_CAP][4] = {};   // row i - 1: this lane's rows of Dinv and the upper blocks
    bool have_prev = false;
    unsigned fl = 0;
    int4 rc[6];
    load_rec(rec, R, c, nch, 0, rc);
    for (int t = 0; t < m; ++t) {
        const int i = c0 + t;
        const int b0 = rec_field<0>(rc), lb = rec_field<1>(rc), ub = rec_field<2>(rc), meta = rec_field<3>(rc);
        const int nl = meta & 15, nu = (meta >> 4) & 15, np = (meta >> 8) & 15;
        const int jl[REC_CAP] = {rec_field<4>(rc), rec_field<5>(rc), rec_field<6>(rc), rec_field<7>(rc)};
        const int pc[REC_CAP] = {rec_field<8>(rc), rec_field<9>(rc), rec_field<10>(rc), rec_field<11>(rc)};
        const int sp[REC_CAP] = {rec_field<12>(rc), rec_field<13>(rc), rec_field<14>(rc), rec_field<15>(rc)};
        const int pk[REC_CAP] = {rec_field<16>(rc), rec_field<17>(rc), rec_field<18>(rc), rec_field<19>(rc)};
        if (nl > REC_CAP || nu > REC_CAP || np > REC_CAP) {
            if (t + 1 < m) load_rec(rec, R, c, nch, t + 1, rc);
            factor_chunk_row<T, OUT_FROM_A, true>(i, c0, ubound, n, ZL, rowptr, colidx, diag_pos, lrow, urow,
                                                  pair_ptr, pkj, sik, skj, A, XO, DO, Xn, Dn, flags);
            have_prev = false;
            continue;
        }
        // every operand of the row: A's blocks, the inverses of the lower neighbours, the U_kj
        T aL[REC_CAP][4], aD[4], aU[REC_CAP][4], dj[REC_CAP][4], uv[REC_CAP][4];
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u)
            if (u < nl) load_row(A + (int64_t)(b0 + u) * BB, r, aL[u]);
        load_row(A + (int64_t)(b0 + nl) * BB, r, aD);
#pragma unroll
        for (int w = 0; w < REC_CAP; ++w)
            if (w < nu) load_row(A + (int64_t)(b0 + nl + 1 + w) * BB, r, aU[w]);
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u) {
            if (u < nl) {
                const int src = (meta >> (12 + 2 * u)) & 3;
                if (src == REC_PREV && have_prev) copy_row(pD, dj[u]);
                else load_row((src == REC_OUT ? DO : (const T *)Dn) + (int64_t)jl[u] * BB, r, dj[u]);
            }
        }
#pragma unroll
        for (int q = 0; q < REC_CAP; ++q) {
            if (q < np) {
                const int src = (pc[q] >> 6) & 3;
                if (src == REC_PREV && have_prev) pick_row(pU, (pc[q] >> 8) & 3, uv[q]);
                else if (src != REC_OUT) load_row((const T *)Xn + (int64_t)sp[q] * BB, r, uv[q]);
                else if constexpr (OUT_FROM_A) load_row(A + (int64_t)pk[q] * BB, r, uv[q]);
                else load_row(XO + (int64_t)sp[q] * BB, r, uv[q]);
            }
        }
        if (t + 1 < m) load_rec(rec, R, c, nch, t + 1, rc);   // the next row's record, behind this row's loads
        // strictly lower blocks in ascending column order, each seeing the ones before it
        T Lx[REC_CAP][4] = {};
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u) {
            if (u < nl) {
                T tt[4];
                copy_row(aL[u], tt);
#pragma unroll
                for (int q = 0; q < REC_CAP; ++q) {
                    if (q < np && (pc[q] & 15) == u) {
                        T l[4];
                        pick_row(Lx, (pc[q] >> 4) & 3, l);
                        row_times_block_sub(l, uv[q], tt);
                    }
                }
                row_times_block(tt, dj[u], Lx[u]);
                fl |= nonfinite4(Lx[u]);
                store_row(Xn + ((int64_t)lb + u) * BB, r, Lx[u]);
            }
        }
        // diagonal block and its inverse
        {
#pragma unroll
            for (int q = 0; q < REC_CAP; ++q) {
                if (q < np && (pc[q] & 15) == 4) {
                    T l[4];
                    pick_row(Lx, (pc[q] >> 4) & 3, l);
                    row_times_block_sub(l, uv[q], aD);
                }
            }
            fl |= nonfinite4(aD);
            store_row(Xn + ((int64_t)ZL + i) * BB, r, aD);
            T M[16];
            gather_block(aD, M);
            if (!inv4_row(M, r, pD)) fl |= ABILU_FLAG_MODIFIED;
            store_row(Dn + (int64_t)i * BB, r, pD);
        }
        // strictly upper blocks
#pragma unroll
        for (int w = 0; w < REC_CAP; ++w) {
            if (w < nu) {
#pragma unroll
                for (int q = 0; q < REC_CAP; ++q) {
                    if (q < np && (pc[q] & 15) == 5 + w) {
                        T l[4];
                        pick_row(Lx, (pc[q] >> 4) & 3, l);
                        row_times_block_sub(l, uv[q], aU[w]);
                    }
                }
                fl |= nonfinite4(aU[w]);
                store_row(Xn + ((int64_t)ubase + ub + w) * BB, r, aU[w]);
                copy_row(aU[w], pU[w]);
            }
        }
        have_prev = true;
    }
    if (fl) atomicOr(flags, fl);
}

// Pipelined form of the record runner, for patterns whose every row holds at most CL strictly lower
// and CU strictly upper blocks and CP update pairs: row i + 1's operands are fetched while row i is
// computed, so the chunk's chain of rows overlaps each row's memory round trip with the previous
// row's arithmetic. The fetched operands are held as loaded (A's blocks in FP64, converted when
// used) so that no instruction waits for them before the row that uses them. The row computed
// just before supplies its values from registers. The arithmetic and its order are those of
// factor_chunk_row.
template <int CL, int CP>
struct RecRow {
    int b0, lb, ub, meta, nl, nu, np;
    int jl[CL], pc[CP], sp[CP], pk[CP];
};

template <int CL, int CP>
__device__ __forceinline__ RecRow<CL, CP> decode_rec(const int4 (&rc)[6]) {
    const int v[20] = {rec_field<0>(rc),  rec_field<1>(rc),  rec_field<2>(rc),  rec_field<3>(rc),  rec_field<4>(rc),
                       rec_field<5>(rc),  rec_field<6>(rc),  rec_field<7>(rc),  rec_field<8>(rc),  rec_field<9>(rc),
                       rec_field<10>(rc), rec_field<11>(rc), rec_field<12>(rc), rec_field<13>(rc), rec_field<14>(rc),
                       rec_field<15>(rc), rec_field<16>(rc), rec_field<17>(rc), rec_field<18>(rc), rec_field<19>(rc)};
    RecRow<CL, CP> f;
    f.b0 = v[0];
    f.lb = v[1];
    f.ub = v[2];
    f.meta = v[3];
    f.nl = f.meta & 15;
    f.nu = (f.meta >> 4) & 15;
    f.np = (f.meta >> 8) & 15;
#pragma unroll
    for (int u = 0; u < CL; ++u) f.jl[u] = v[4 + u];
#pragma unroll
    for (int q = 0; q < CP; ++q) {
        f.pc[q] = v[8 + q];
        f.sp[q] = v[12 + q];
        f.pk[q] = v[16 + q];
    }
    return f;
}

template <typename T, bool OUT_FROM_A, int CL, int CU, int CP>
struct RowOps {
    double aL[CL][4], aD[4], aU[CU][4];           // A's blocks as stored
    T dj[CL][4];                                  // inverses of the lower neighbours
    T uv[CP][4];                                  // U_kj from the factor
    double ua[OUT_FROM_A ? CP : 1][4];            // U_kj from A (first sweep, rows outside the chunk)
};

template <typename T, bool OUT_FROM_A, int CL, int CU, int CP>
__device__ __forceinline__ void issue_row(const RecRow<CL, CP> &f, int r, const double *__restrict__ A, const T *XO,
                                          const T *DO, const T *Xn, const T *Dn,
                                          RowOps<T, OUT_FROM_A, CL, CU, CP> &o) {
    // A's blocks, clamped to the row (an unused slot re-reads the diagonal block)
#pragma unroll
    for (int u = 0; u < CL; ++u) load_row(A + (int64_t)(f.b0 + min(u, f.nl)) * BB, r, o.aL[u]);
    load_row(A + (int64_t)(f.b0 + f.nl) * BB, r, o.aD);
#pragma unroll
    for (int w = 0; w < CU; ++w) load_row(A + (int64_t)(f.b0 + f.nl + min(w + 1, f.nu)) * BB, r, o.aU[w]);
#pragma unroll
    for (int u = 0; u < CL; ++u) {
        const int src = (f.meta >> (12 + 2 * u)) & 3;
        if (u < f.nl && src != REC_PREV) load_row((src == REC_OUT ? DO : Dn) + (int64_t)f.jl[u] * BB, r, o.dj[u]);
    }
#pragma unroll
    for (int q = 0; q < CP; ++q) {
        const int src = (f.pc[q] >> 6) & 3;
        if (q < f.np && src != REC_PREV) {
            if constexpr (OUT_FROM_A) {
                if (src == REC_CHUNK) load_row(Xn + (int64_t)f.sp[q] * BB, r, o.uv[q]);
                else load_row(A + (int64_t)f.pk[q] * BB, r, o.ua[q]);
            } else {
                load_row((src == REC_OUT ? XO : Xn) + (int64_t)f.sp[q] * BB, r, o.uv[q]);
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ void to_t(const double (&a)[4], T (&v)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (T)a[c];
}

template <typename T, bool OUT_FROM_A, int CL, int CU, int CP>
__device__ __forceinline__ unsigned compute_row(const RecRow<CL, CP> &f, int i, int r, int ZL, int ubase,
                                                const RowOps<T, OUT_FROM_A, CL, CU, CP> &o, T (&pD)[4],
                                                T (&pU)[CU][4], T *Xn, T *Dn) {
    unsigned fl = 0;
    T dj[CL][4], uq[CP][4];
#pragma unroll
    for (int u = 0; u < CL; ++u) {
        if (u < f.nl) {
            if (((f.meta >> (12 + 2 * u)) & 3) != REC_PREV) copy_row(o.dj[u], dj[u]);
            else copy_row(pD, dj[u]);
        }
    }
#pragma unroll
    for (int q = 0; q < CP; ++q) {
        if (q < f.np) {
            const int src = (f.pc[q] >> 6) & 3;
            if (src == REC_PREV) pick_row(pU, (f.pc[q] >> 8) & 3, uq[q]);
            else if constexpr (OUT_FROM_A) {
                if (src == REC_OUT) to_t(o.ua[q], uq[q]);
                else copy_row(o.uv[q], uq[q]);
            } else {
                copy_row(o.uv[q], uq[q]);
            }
        }
    }
    // strictly lower blocks in ascending column order, each seeing the ones before it
    T Lx[CL][4] = {};
#pragma unroll
    for (int u = 0; u < CL; ++u) {
        if (u < f.nl) {
            T tt[4];
            to_t(o.aL[u], tt);
#pragma unroll
            for (int q = 0; q < CP; ++q) {
                if (q < f.np && (f.pc[q] & 15) == u) {
                    T l[4];
                    pick_row(Lx, (f.pc[q] >> 4) & 3, l);
                    row_times_block_sub(l, uq[q], tt);
                }
            }
            row_times_block(tt, dj[u], Lx[u]);
            fl |= nonfinite4(Lx[u]);
            store_row(Xn + ((int64_t)f.lb + u) * BB, r, Lx[u]);
        }
    }
    // diagonal block and its inverse
    {
        T td[4];
        to_t(o.aD, td);
#pragma unroll
        for (int q = 0; q < CP; ++q) {
            if (q < f.np && (f.pc[q] & 15) == 4) {
                T l[4];
                pick_row(Lx, (f.pc[q] >> 4) & 3, l);
                row_times_block_sub(l, uq[q], td);
            }
        }
        fl |= nonfinite4(td);
        store_row(Xn + ((int64_t)ZL + i) * BB, r, td);
        T M[16];
        gather_block(td, M);
        if (!inv4_row(M, r, pD)) fl |= ABILU_FLAG_MODIFIED;
        store_row(Dn + (int64_t)i * BB, r, pD);
    }
    // strictly upper blocks
#pragma unroll
    for (int w = 0; w < CU; ++w) {
        if (w < f.nu) {
            T tt[4];
            to_t(o.aU[w], tt);
#pragma unroll
            for (int q = 0; q < CP; ++q) {
                if (q < f.np && (f.pc[q] & 15) == 5 + w) {
                    T l[4];
                    pick_row(Lx, (f.pc[q] >> 4) & 3, l);
                    row_times_block_sub(l, uq[q], tt);
                }
            }
            fl |= nonfinite4(tt);
            store_row(Xn + ((int64_t)ubase + f.ub + w) * BB, r, tt);
            copy_row(tt, pU[w]);
        }
    }
    return fl;
}

template <typename T, bool OUT_FROM_A, int CL, int CU, int CP>
__global__ __launch_bounds__(WG) void k_factor_sweep_chunk_rows_pipe(int n, int ZL, int R, int nch,
                                                                     const int32_t *__restrict__ rec,
                                                                     const double *__restrict__ A, const T *XO,
                                                                     const T *DO, T *Xn, T *Dn, unsigned *flags) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    if (c >= nch) return;
    const int r = threadIdx.x & 3;
    const int c0 = c * R, m = min(n, c0 + R) - c0;
    const int ubase = ZL + n;
    T pD[4] = {}, pU[CU][4] = {};   // row i - 1: this lane's rows of Dinv and the upper blocks
    unsigned fl = 0;
    int4 rc[6];
    load_rec(rec, R, c, nch, 0, rc);
    RecRow<CL, CP> f0 = decode_rec<CL, CP>(rc), f1 = f0;
    RowOps<T, OUT_FROM_A, CL, CU, CP> o0, o1;
    issue_row<T, OUT_FROM_A>(f0, r, A, XO, DO, Xn, Dn, o0);
    if (m > 1) load_rec(rec, R, c, nch, 1, rc);
    // row t from (fc, oc); row t + 1 fetched into (fn, on) first
    auto step = [&](int t, const RecRow<CL, CP> &fc, const RowOps<T, OUT_FROM_A, CL, CU, CP> &oc,
                    RecRow<CL, CP> &fn, RowOps<T, OUT_FROM_A, CL, CU, CP> &on) {
        if (t + 1 < m) {
            fn = decode_rec<CL, CP>(rc);
            issue_row<T, OUT_FROM_A>(fn, r, A, XO, DO, Xn, Dn, on);
            if (t + 2 < m) load_rec(rec, R, c, nch, t + 2, rc);
        }
        fl |= compute_row<T, OUT_FROM_A>(fc, c0 + t, r, ZL, ubase, oc, pD, pU, Xn, Dn);
    };
    for (int t = 0; t < m; t += 2) {
        step(t, f0, o0, f1, o1);
        if (t + 1 < m) step(t + 1, f1, o1, f0, o0);
    }
    if (fl) atomicOr(flags, fl);
}

// Conversions between the factor layout and CSR order (one quad per block row).
template <typename T, bool TO_CSR>
__global__ __launch_bounds__(WG) void k_factor_permute(int n, int ZL, const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ diag_pos,
                                                       const int32_t *__restrict__ lrow,
                                                       const int32_t *__restrict__ urow, const T *__restrict__ src,
                                                       T *__restrict__ dst) {
    const int i = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    const int r = threadIdx.x & 3;
    if (i >= n) return;
    const int b0 = rowptr[i], d = diag_pos[i], b1 = rowptr[i + 1];
    for (int e = b0; e < b1; ++e) {
        const int64_t sp = split_pos(e, i, b0, d, lrow[i], urow[i], ZL, n);
        T v[4];
        load_row(src + (TO_CSR ? sp : (int64_t)e) * BB, r, v);
        store_row(dst + (TO_CSR ? (int64_t)e : sp) * BB, r, v);
    }
}

template <typename T>
const char *tname();
template <>
const char *tname<float>() { return "f32"; }
template <>
const char *tname<double>() { return "f64"; }

template <typename T, bool LA, bool UA, bool DA = false>
void launch_sweep(const abilu_pattern *p, int grid, hipStream_t s, const double *A, const T *XL, const T *XU,
                  const T *Dp, T *Xn, T *Dn, unsigned *flags) {
    k_factor_sweep<T, LA, UA, DA><<<grid, WG, 0, s>>>(p->n, (int)p->nnzb_lower, p->rowptr, p->colidx, p->diag_pos,
                                                       p->lrow, p->urow, p->pair_ptr, p->pik, p->pkj, p->sik, p->skj,
                                                       A, XL, XU, Dp, Xn, Dn, flags, p->symmetric ? 1 : 0);
}

template <typename T>
abilu_status factor_t(const abilu_pattern *p, const double *A, T *LU, T *Dinv, int nsw, abilu_mode mode,
                      abilu_init init, char *work, const Workspace &W, hipStream_t s) {
    const int n = p->n;
    const int ZL = (int)p->nnzb_lower;
    const int grid = div_up(n, ROWS_PER_WG);
    unsigned *flags = (unsigned *)(work + W.flags);
    T *X1 = (T *)(work + W.x2);
    T *D1 = (T *)(work + W.d2);
    char name[64];
    auto NAME = [&](const char *base, const char *suffix) {
        snprintf(name, sizeof name, "%s_%s%s", base, tname<T>(), suffix);
        return name;
    };
    const Sizes z = sizes(p);
    const double sF = sizeof(T);
#define LAUNCHED() \
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE

    auto init_dinv_A = [&](T *D0) -> abilu_status {
        ProfScope ps(NAME("factor_init", ""), s, bytes_init(z, 8, sF, false));
        k_factor_init<T, double, true, false><<<grid, WG, 0, s>>>(n, ZL, p->rowptr, p->diag_pos, p->lrow, p->urow, A,
                                                                  (T *)nullptr, D0, flags);
        LAUNCHED();
        return ABILU_OK;
    };
    auto init_dinv_X = [&](const T *X0, T *D0) -> abilu_status {
        ProfScope ps(NAME("factor_init", ""), s, bytes_init(z, sF, sF, false));
        k_factor_init<T, T, false, false><<<grid, WG, 0, s>>>(n, ZL, p->rowptr, p->diag_pos, p->lrow, p->urow, X0,
                                                              (T *)nullptr, D0, flags);
        LAUNCHED();
        return ABILU_OK;
    };
    abilu_status st;

    if (nsw == 0) {
        if (init == ABILU_INIT_FROM_A) {
            ProfScope ps(NAME("factor_init", "_copy"), s, bytes_init(z, 8, sF, true));
            k_factor_init<T, double, true, true><<<grid, WG, 0, s>>>(n, ZL, p->rowptr, p->diag_pos, p->lrow, p->urow,
                                                                     A, LU, Dinv, flags);
            LAUNCHED();
            return ABILU_OK;
        }
        return init_dinv_X(LU, Dinv);
    }

    if (mode == ABILU_ASYNC_SERIAL) {
        // X0 copied into LU (from A) or taken from LU, then nsw in-place sweeps by one worker
        if (init == ABILU_INIT_FROM_A) {
            ProfScope ps(NAME("factor_init", "_copy"), s, bytes_init(z, 8, sF, true));
            k_factor_init<T, double, true, true><<<grid, WG, 0, s>>>(n, ZL, p->rowptr, p->diag_pos, p->lrow, p->urow,
                                                                     A, LU, Dinv, flags);
            LAUNCHED();
        } else if ((st = init_dinv_X(LU, Dinv)) != ABILU_OK) {
            return st;
        }
        for (int q = 0; q < nsw; ++q) {
            ProfScope ps(NAME("factor_sweep", "_serial"), s, bytes_sweep(z, sF, false, false));
            k_factor_sweep_serial<T><<<1, 4, 0, s>>>(n, ZL, p->rowptr, p->colidx, p->diag_pos, p->lrow, p->urow,
                                                     p->pair_ptr, p->pik, p->pkj, p->sik, p->skj, A, LU, Dinv, flags);
            LAUNCHED();
        }
        return ABILU_OK;
    }

    if (mode == ABILU_CHUNK_SYNC || mode == ABILU_CHUNK_ASYNC) {
        // Chunked sweeps. CHUNK_SYNC reads other chunks from the previous sweep (ping-pong as in
        // SYNC); CHUNK_ASYNC works in place. The first sweep from A reads other chunks' blocks
        // from A itself (X0) in both modes.
        const bool cs = (mode == ABILU_CHUNK_SYNC);
        const double sched = 4.0 * z.N + 4.0 * (p->nchunks + 1) + 4.0 * (double)(p->total_levels[0] + p->nchunks);
        auto chunk_sweep = [&](bool fromA, const T *XO, const T *DO, T *Xn, T *Dn, const char *nm) -> abilu_status {
            ProfScope ps(NAME("factor_sweep", nm), s, bytes_sweep(z, sF, false, fromA) + sched);
            if (p->chunk_runner == ABILU_CHUNK_BY_ROWS) {
                const int g = div_up(p->nchunks, ROWS_PER_WG);
                // the pipelined form in FP32 when every row of the pattern fits its capacities (2 lower
                // and 2 upper blocks, 2 update pairs; in FP64 two rows' operands exceed the register
                // file), otherwise the general record runner
                bool pipelined = false;
                if constexpr (sizeof(T) == 4) {
                    if (p->rec_max[0] <= 2 && p->rec_max[1] <= 2 && p->rec_max[2] <= 2) {
                        if (fromA)
                            k_factor_sweep_chunk_rows_pipe<T, true, 2, 2, 2><<<g, WG, 0, s>>>(
                                n, ZL, p->chunk_rows, p->nchunks, p->rec, A, XO, DO, Xn, Dn, flags);
                        else
                            k_factor_sweep_chunk_rows_pipe<T, false, 2, 2, 2><<<g, WG, 0, s>>>(
                                n, ZL, p->chunk_rows, p->nchunks, p->rec, A, XO, DO, Xn, Dn, flags);
                        pipelined = true;
                    }
                }
#define ABILU_CHUNK_ROWS_ARGS                                                                                \
    n, ZL, p->chunk_rows, p->nchunks, p->rec, p->rowptr, p->colidx, p->diag_pos, p->lrow, p->urow, p->pair_ptr, \
        p->pkj, p->sik, p->skj, A, XO, DO, Xn, Dn, flags
                if (!pipelined && fromA)
                    k_factor_sweep_chunk_rows<T, true><<<g, WG, 0, s>>>(ABILU_CHUNK_ROWS_ARGS);
                else if (!pipelined)
                    k_factor_sweep_chunk_rows<T, false><<<g, WG, 0, s>>>(ABILU_CHUNK_ROWS_ARGS);
#undef ABILU_CHUNK_ROWS_ARGS
            } else if (fromA)
                k_factor_sweep_chunk<T, true><<<p->nchunks, WG, 0, s>>>(
                    n, ZL, p->chunk_rows, p->order[0], p->lvptr[0], p->lvstart[0], p->rowptr, p->colidx, p->diag_pos,
                    p->lrow, p->urow, p->pair_ptr, p->pkj, p->sik, p->skj, A, XO, DO, Xn, Dn, flags);
            else
                k_factor_sweep_chunk<T, false><<<p->nchunks, WG, 0, s>>>(
                    n, ZL, p->chunk_rows, p->order[0], p->lvptr[0], p->lvstart[0], p->rowptr, p->colidx, p->diag_pos,
                    p->lrow, p->urow, p->pair_ptr, p->pkj, p->sik, p->skj, A, XO, DO, Xn, Dn, flags);
            LAUNCHED();
            return ABILU_OK;
        };
        if (!cs) {
            int q0 = 0;
            if (init == ABILU_INIT_FROM_A) {
                if ((st = init_dinv_A(Dinv)) != ABILU_OK) return st;
                if ((st = chunk_sweep(true, (const T *)nullptr, Dinv, LU, Dinv, "_chunk_async_fromA")) != ABILU_OK)
                    return st;
                q0 = 1;
            } else if ((st = init_dinv_X(LU, Dinv)) != ABILU_OK) {
                return st;
            }
            for (int q = q0; q < nsw; ++q)
                if ((st = chunk_sweep(false, LU, Dinv, LU, Dinv, "_chunk_async")) != ABILU_OK) return st;
            return ABILU_OK;
        }
        auto cX = [&](int q) { return ((nsw - q) % 2 == 0) ? LU : X1; };
        auto cD = [&](int q) { return ((nsw - q) % 2 == 0) ? Dinv : D1; };
        if (init == ABILU_INIT_FROM_A) {
            if ((st = init_dinv_A(cD(0))) != ABILU_OK) return st;
            if ((st = chunk_sweep(true, (const T *)nullptr, cD(0), cX(1), cD(1), "_chunk_sync_fromA")) != ABILU_OK)
                return st;
        } else {
            T *X0 = LU;
            if (cX(1) == LU) {
                if (!hip_ok(hipMemcpyAsync(X1, LU, sizeof(T) * BB * (size_t)p->nnzb, hipMemcpyDeviceToDevice, s),
                            "warm-start copy"))
                    return ABILU_EDEVICE;
                X0 = X1;
            }
            if ((st = init_dinv_X(X0, cD(0))) != ABILU_OK) return st;
            if ((st = chunk_sweep(false, X0, cD(0), cX(1), cD(1), "_chunk_sync")) != ABILU_OK) return st;
        }
        for (int q = 2; q <= nsw; ++q)
            if ((st = chunk_sweep(false, cX(q - 1), cD(q - 1), cX(q), cD(q), "_chunk_sync")) != ABILU_OK) return st;
        return ABILU_OK;
    }

    if (mode == ABILU_ASYNC) {
        int q0 = 0;
        if (init == ABILU_INIT_FROM_A) {
            // the first sweep forms the initial inverses inv(A_jj) itself (no initialisation pass)
            ProfScope ps(NAME("factor_sweep", "_async_fromA"), s, bytes_sweep_from_a(z, sF, false));
            launch_sweep<T, false, true, true>(p, grid, s, A, LU, (const T *)nullptr, Dinv, LU, Dinv, flags);
            LAUNCHED();
            q0 = 1;
        } else if ((st = init_dinv_X(LU, Dinv)) != ABILU_OK) {
            return st;
        }
        for (int q = q0; q < nsw; ++q) {
            ProfScope ps(NAME("factor_sweep", "_async"), s, bytes_sweep(z, sF, false, false));
            launch_sweep<T, false, false>(p, grid, s, A, LU, LU, Dinv, LU, Dinv, flags);
            LAUNCHED();
        }
        return ABILU_OK;
    }

    // SYNC with nsw >= 1: sweep q (1-based) writes buffer out(q); out(nsw) is the caller's.
    auto outX = [&](int q) { return ((nsw - q) % 2 == 0) ? LU : X1; };
    auto outD = [&](int q) { return ((nsw - q) % 2 == 0) ? Dinv : D1; };
    T *D0 = outD(0);
    if (init == ABILU_INIT_FROM_A) {
        // the first sweep forms the initial inverses inv(A_jj) itself (no initialisation pass)
        ProfScope ps(NAME("factor_sweep", "_sync_fromA"), s, bytes_sweep_from_a(z, sF, true));
        launch_sweep<T, true, true, true>(p, grid, s, A, (const T *)nullptr, (const T *)nullptr, D0, outX(1),
                                          outD(1), flags);
        LAUNCHED();
    } else {
        // warm start: X0 = d_LU. Sweep 1 must not write where it reads.
        T *X0 = LU;
        if (outX(1) == LU) {
            if (!hip_ok(hipMemcpyAsync(X1, LU, sizeof(T) * BB * (size_t)p->nnzb, hipMemcpyDeviceToDevice, s),
                        "warm-start copy"))
                return ABILU_EDEVICE;
            X0 = X1;
        }
        if ((st = init_dinv_X(X0, D0)) != ABILU_OK) return st;
        ProfScope ps(NAME("factor_sweep", "_sync"), s, bytes_sweep(z, sF, false, false));
        launch_sweep<T, false, false>(p, grid, s, A, X0, X0, D0, outX(1), outD(1), flags);
        LAUNCHED();
    }
    for (int q = 2; q <= nsw; ++q) {
        ProfScope ps(NAME("factor_sweep", "_sync"), s, bytes_sweep(z, sF, false, false));
        launch_sweep<T, false, false>(p, grid, s, A, outX(q - 1), outX(q - 1), outD(q - 1), outX(q), outD(q), flags);
        LAUNCHED();
    }
    return ABILU_OK;
#undef LAUNCHED
}

template <typename T>
abilu_status permute_t(const abilu_pattern *p, const T *src, T *dst, bool to_csr, hipStream_t s) {
    const int grid = div_up(p->n, ROWS_PER_WG);
    const int ZL = (int)p->nnzb_lower;
    ProfScope ps(to_csr ? "factor_to_csr" : "factor_from_csr", s, 2.0 * 16 * sizeof(T) * (double)p->nnzb);
    if (to_csr)
        k_factor_permute<T, true><<<grid, WG, 0, s>>>(p->n, ZL, p->rowptr, p->diag_pos, p->lrow, p->urow, src, dst);
    else
        k_factor_permute<T, false><<<grid, WG, 0, s>>>(p->n, ZL, p->rowptr, p->diag_pos, p->lrow, p->urow, src, dst);
    return launch_status();
}

}  // namespace

extern "C" abilu_status abilu_factor(const abilu_pattern *p, const double *d_A, void *d_LU, void *d_Dinv,
                                     abilu_prec prec, int32_t nsweeps, abilu_mode mode, abilu_init init,
                                     void *d_work, size_t work_bytes, void *stream) {
    if (!p || nsweeps < 0) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    if (!mode_ok(p, mode)) return ABILU_EINVAL;
    if (init != ABILU_INIT_FROM_A && init != ABILU_INIT_FROM_LU) return ABILU_EINVAL;
    if (!d_work) return ABILU_EINVAL;
    const Workspace W = layout(p, prec, 0);
    if (work_bytes < W.total) return ABILU_EINVAL;
    if (p->n == 0) return ABILU_OK;
    if (!d_A || !d_LU || !d_Dinv) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (prec == ABILU_F32)
        return factor_t<float>(p, d_A, (float *)d_LU, (float *)d_Dinv, nsweeps, mode, init, (char *)d_work, W, s);
    return factor_t<double>(p, d_A, (double *)d_LU, (double *)d_Dinv, nsweeps, mode, init, (char *)d_work, W, s);
}

extern "C" abilu_status abilu_factor_to_csr(const abilu_pattern *p, abilu_prec prec, const void *d_LU,
                                            void *d_csr, void *stream) {
    if (!p || (prec != ABILU_F32 && prec != ABILU_F64)) return ABILU_EINVAL;
    if (p->n == 0) return ABILU_OK;
    if (!d_LU || !d_csr || d_LU == d_csr) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (prec == ABILU_F32) return permute_t<float>(p, (const float *)d_LU, (float *)d_csr, true, s);
    return permute_t<double>(p, (const double *)d_LU, (double *)d_csr, true, s);
}

extern "C" abilu_status abilu_factor_from_csr(const abilu_pattern *p, abilu_prec prec, const void *d_csr,
                                              void *d_LU, void *stream) {
    if (!p || (prec != ABILU_F32 && prec != ABILU_F64)) return ABILU_EINVAL;
    if (p->n == 0) return ABILU_OK;
    if (!d_LU || !d_csr || d_LU == d_csr) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (prec == ABILU_F32) return permute_t<float>(p, (const float *)d_csr, (float *)d_LU, false, s);
    return permute_t<double>(p, (const double *)d_csr, (double *)d_LU, false, s);
}
