// Block ILU(0) factorisation sweeps (Section 4.2).
//
// Every block (i,j) of S_B is an unknown of the fixed-point equations (equation blockH):
//   H_ij(X) = (A_ij - sum_{k in K(i,j)} X_ik X_kj) X_jj^{-1}   for i > j
//   H_ij(X) =  A_ij - sum_{k in K(i,j)} X_ik X_kj              for i <= j
// One sweep evaluates H for every block at once. The diagonal inverses are carried as a second
// array Dinv (the exact 4x4 inversion of each diagonal block, fused into the sweep: the quad
// that produces U_ii inverts it on the spot).
//
// Mapping: one quad of 4 lanes per block row i; lane r owns row r of every 4x4 block of the row
// (so a block is one contiguous 64/128-byte access by the quad) and rows of other blocks are
// exchanged inside the quad by DPP broadcasts. 64 block rows per 256-thread workgroup; the
// workgroup index is remapped so each XCD sweeps one contiguous range of rows.
//
// SYNC: reads only X^p, Dinv^p and writes X^{p+1}, Dinv^{p+1} (ping-pong buffers): the
//       Jacobi-type iteration x^{p+1} = h(x^p). Deterministic.
// ASYNC: X and Dinv are updated in place; reads see whatever value is in memory (possibly a
//       block that another quad is writing: torn reads are allowed because each scalar has its
//       own delay in the block-asynchronous model). Within a row the blocks are visited in
//       ascending column order, so U_ii uses the L_ik just computed by the same quad. Sums are
//       accumulated in registers and stored once; no atomics on factor values.
#include "abilu_internal.h"

using namespace abilu;
using namespace abilu_dev;

namespace {

// X0 -> (optional) copy into Xout in precision T, and D0 = inverses of X0's diagonal blocks.
template <typename T, typename S, bool COPY>
__global__ __launch_bounds__(WG) void k_factor_init(int n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ diag_pos,
                                                    const S *X0, T *Xout, T *D0, unsigned *flags) {
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int i = wg * ROWS_PER_WG + (threadIdx.x >> 2);
    const int r = threadIdx.x & 3;
    if (i >= n) return;
    const int d = diag_pos[i];
    if constexpr (COPY) {
        const int b0 = rowptr[i], b1 = rowptr[i + 1];
        for (int e = b0; e < b1; ++e) {
            T v[4];
            load_row(X0 + (int64_t)e * BB, r, v);
            store_row(Xout + (int64_t)e * BB, r, v);
        }
    }
    T u[4], M[16], R[16], out[4];
    load_row(X0 + (int64_t)d * BB, r, u);
    gather_block(u, M);
    bool ok = inv4(M, R);
    pick_row(R, r, out);
    store_row(D0 + (int64_t)i * BB, r, out);
    if (!ok && r == 0) atomicOr(flags, ABILU_FLAG_MODIFIED);
}

// t -= sum over the update set of block e of X_ik X_kj (this lane's row of the product)
template <typename T, typename S>
__device__ __forceinline__ void update_terms(int e, int r, const int32_t *__restrict__ pair_ptr,
                                             const int32_t *__restrict__ pik,
                                             const int32_t *__restrict__ pkj, const S *Xp, T (&t)[4]) {
    const int p0 = pair_ptr[e], p1 = pair_ptr[e + 1];
    for (int p = p0; p < p1; ++p) {
        const int ik = pik[p], kj = pkj[p];
        T l[4], u[4];
        load_row(Xp + (int64_t)ik * BB, r, l);
        load_row(Xp + (int64_t)kj * BB, r, u);
        row_times_block_sub(l, u, t);
    }
}

// One sweep. S = element type of the iterate read (double when the iterate is A itself).
template <typename T, typename S>
__global__ __launch_bounds__(WG) void k_factor_sweep(
    int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ pair_ptr,
    const int32_t *__restrict__ pik, const int32_t *__restrict__ pkj, const double *__restrict__ A,
    const S *Xp, const T *Dp, T *Xn, T *Dn, unsigned *flags) {
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int i = wg * ROWS_PER_WG + (threadIdx.x >> 2);
    const int r = threadIdx.x & 3;
    if (i >= n) return;
    const int b0 = rowptr[i], b1 = rowptr[i + 1], d = diag_pos[i];
    unsigned fl = 0;
    // strictly lower blocks: L_ij = (A_ij - sum) U_jj^{-1}
    for (int e = b0; e < d; ++e) {
        T t[4];
        load_row(A + (int64_t)e * BB, r, t);
        update_terms(e, r, pair_ptr, pik, pkj, Xp, t);
        const int j = colidx[e];
        T dr[4], x[4];
        load_row(Dp + (int64_t)j * BB, r, dr);
        row_times_block(t, dr, x);
        fl |= nonfinite4(x);
        store_row(Xn + (int64_t)e * BB, r, x);
    }
    // diagonal block U_ii = A_ii - sum, and its inverse
    {
        T t[4];
        load_row(A + (int64_t)d * BB, r, t);
        update_terms(d, r, pair_ptr, pik, pkj, Xp, t);
        fl |= nonfinite4(t);
        store_row(Xn + (int64_t)d * BB, r, t);
        T M[16], R[16], out[4];
        gather_block(t, M);
        if (!inv4(M, R)) fl |= ABILU_FLAG_MODIFIED;
        pick_row(R, r, out);
        store_row(Dn + (int64_t)i * BB, r, out);
    }
    // strictly upper blocks: U_ij = A_ij - sum
    for (int e = d + 1; e < b1; ++e) {
        T t[4];
        load_row(A + (int64_t)e * BB, r, t);
        update_terms(e, r, pair_ptr, pik, pkj, Xp, t);
        fl |= nonfinite4(t);
        store_row(Xn + (int64_t)e * BB, r, t);
    }
    if (fl) atomicOr(flags, fl);
}

template <typename T>
const char *tname();
template <>
const char *tname<float>() { return "f32"; }
template <>
const char *tname<double>() { return "f64"; }

// Algorithmic bytes of one launch: every array element touched once.
// init with copy: rowptr, diag_pos, A (f64), X0 written, Dinv written
// init without copy: diag_pos, diagonal blocks of the source, Dinv written
double bytes_init(const Sizes &z, double sS, double sF, bool copy) {
    if (copy) return 4 * (z.N + 1) + 4 * z.N + 128 * z.Z + 16 * sF * z.Z + 16 * sF * z.N;
    return 4 * z.N + 16 * sS * z.N + 16 * sF * z.N;
}
// sweep: rowptr, diag_pos, colidx of strictly lower blocks, pair_ptr, pair lists, A (f64),
// the blocks the update sets read (min(2P, Z) of them; none extra when they are A's own),
// Dinv read, X written, Dinv written
double bytes_sweep(const Sizes &z, double sF, bool fromA) {
    const double xr = fromA ? 0.0 : 16 * sF * (2 * z.P < z.Z ? 2 * z.P : z.Z);
    return 4 * (z.N + 1) + 4 * z.N + 4 * z.ZL + 4 * (z.Z + 1) + 8 * z.P + 128 * z.Z + xr + 16 * sF * z.N +
           16 * sF * z.Z + 16 * sF * z.N;
}

template <typename T>
abilu_status factor_t(const abilu_pattern *p, const double *A, T *LU, T *Dinv, int nsw, abilu_mode mode,
                      abilu_init init, char *work, const Workspace &W, hipStream_t s) {
    const int n = p->n;
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

    if (mode == ABILU_ASYNC || nsw == 0) {
        // X0 in d_LU, D0 in d_Dinv, then in-place sweeps
        if (init == ABILU_INIT_FROM_A) {
            ProfScope ps(NAME("factor_init", "_copy"), s, bytes_init(z, 8, sF, true));
            k_factor_init<T, double, true><<<grid, WG, 0, s>>>(n, p->rowptr, p->diag_pos, A, LU, Dinv, flags);
        } else {
            ProfScope ps(NAME("factor_init", ""), s, bytes_init(z, sF, sF, false));
            k_factor_init<T, T, false><<<grid, WG, 0, s>>>(n, p->rowptr, p->diag_pos, LU, (T *)nullptr, Dinv, flags);
        }
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
        for (int q = 0; q < nsw; ++q) {
            ProfScope ps(NAME("factor_sweep", "_async"), s, bytes_sweep(z, sF, false));
            k_factor_sweep<T, T><<<grid, WG, 0, s>>>(n, p->rowptr, p->colidx, p->diag_pos, p->pair_ptr, p->pik,
                                                     p->pkj, A, LU, Dinv, LU, Dinv, flags);
            if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
        }
        return ABILU_OK;
    }

    // SYNC with nsw >= 1: sweep q (1-based) writes buffer out(q); out(nsw) is the caller's.
    auto outX = [&](int q) { return ((nsw - q) % 2 == 0) ? LU : X1; };
    auto outD = [&](int q) { return ((nsw - q) % 2 == 0) ? Dinv : D1; };
    T *D0 = outD(0);
    if (init == ABILU_INIT_FROM_A) {
        {
            ProfScope ps(NAME("factor_init", ""), s, bytes_init(z, 8, sF, false));
            k_factor_init<T, double, false><<<grid, WG, 0, s>>>(n, p->rowptr, p->diag_pos, A, (T *)nullptr, D0, flags);
        }
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
        {
            ProfScope ps(NAME("factor_sweep", "_sync_fromA"), s, bytes_sweep(z, sF, true));
            k_factor_sweep<T, double><<<grid, WG, 0, s>>>(n, p->rowptr, p->colidx, p->diag_pos, p->pair_ptr,
                                                          p->pik, p->pkj, A, A, D0, outX(1), outD(1), flags);
        }
    } else {
        // warm start: X0 = d_LU. Sweep 1 must not write where it reads.
        T *X0 = LU;
        if (outX(1) == LU) {
            if (!hip_ok(hipMemcpyAsync(X1, LU, sizeof(T) * BB * (size_t)p->nnzb, hipMemcpyDeviceToDevice, s),
                        "warm-start copy"))
                return ABILU_EDEVICE;
            X0 = X1;
        }
        {
            ProfScope ps(NAME("factor_init", ""), s, bytes_init(z, sF, sF, false));
            k_factor_init<T, T, false><<<grid, WG, 0, s>>>(n, p->rowptr, p->diag_pos, X0, (T *)nullptr, D0, flags);
        }
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
        {
            ProfScope ps(NAME("factor_sweep", "_sync"), s, bytes_sweep(z, sF, false));
            k_factor_sweep<T, T><<<grid, WG, 0, s>>>(n, p->rowptr, p->colidx, p->diag_pos, p->pair_ptr, p->pik,
                                                     p->pkj, A, X0, D0, outX(1), outD(1), flags);
        }
    }
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    for (int q = 2; q <= nsw; ++q) {
        ProfScope ps(NAME("factor_sweep", "_sync"), s, bytes_sweep(z, sF, false));
        k_factor_sweep<T, T><<<grid, WG, 0, s>>>(n, p->rowptr, p->colidx, p->diag_pos, p->pair_ptr, p->pik, p->pkj,
                                                 A, outX(q - 1), outD(q - 1), outX(q), outD(q), flags);
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    }
    return ABILU_OK;
}

}  // namespace

extern "C" abilu_status abilu_factor(const abilu_pattern *p, const double *d_A, void *d_LU, void *d_Dinv,
                                     abilu_prec prec, int32_t nsweeps, abilu_mode mode, abilu_init init,
                                     void *d_work, size_t work_bytes, void *stream) {
    if (!p || nsweeps < 0) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    if (mode != ABILU_SYNC && mode != ABILU_ASYNC) return ABILU_EINVAL;
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
