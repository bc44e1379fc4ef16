// Restarted flexible GMRES (the Krylov solver of Sections 1 and 6), right-preconditioned by the
// sweep apply, entirely in double precision on the device: Arnoldi basis V and preconditioned
// basis Z in the workspace, classical Gram-Schmidt with a second pass when the norm falls below
// 1/sqrt(2) of its value before orthogonalisation ("twice is enough"), Givens rotations on the
// Hessenberg matrix by one lane of the reduction before them, x update and true residual at each
// cycle end. The host loop reads back a few scalars per iteration to decide when to stop.
//
// All reductions are fixed-order (per-workgroup partials, then one workgroup per column in
// index order), so results do not depend on scheduling. The only atomic is the completion count
// that picks the last workgroup of a reduction; it orders work, not values.
#include <cmath>

#include "kernels.h"

using namespace abilu;
using namespace abilu_dev;
using namespace abilu_k;

namespace {

// partial[k*nb + b] = sum_{t in tile b} V_k[t] w[t] for k < q;  partial[q*nb + b] = sum w[t]^2
__global__ __launch_bounds__(WG) void k_mdot(int64_t len, const double *__restrict__ V, int64_t ldv, int q,
                                             const double *__restrict__ w, double *__restrict__ partial, int nb,
                                             const int *guard) {
    mdot_body(blockIdx.x, len, V, ldv, q, w, partial, nb, guard);
}

// w[t] += alpha * sum_k c[k] V_k[t]; if partial: partial[b] = sum over tile of new w[t]^2. The
// workgroups take the tiles in descending order: the dot products before it run ascending, so it
// starts on the tiles they read last (the partials stay indexed by tile, so sums are unchanged).
__global__ __launch_bounds__(WG) void k_update(int64_t len, const double *__restrict__ V, int64_t ldv, int q,
                                               const double *__restrict__ c, double alpha, double *__restrict__ w,
                                               double *__restrict__ partial, const int *guard) {
    update_body(gridDim.x - 1 - blockIdx.x, len, V, ldv, q, c, alpha, w, partial, guard);
}

// out[col] = sum_b partial[col*nb + b], one workgroup per column, fixed order
__global__ __launch_bounds__(WG) void k_reduce_cols(const double *__restrict__ partial, int nb,
                                                    double *__restrict__ out, const int *guard) {
    reduce_cols_body(blockIdx.x, partial, nb, out, guard);
}

// The single-lane steps that follow a column reduction, run by its last workgroup.
enum { RS_BETA_START_ZERO = 0, RS_BETA_START_X, RS_BETA, RS_GS1, RS_GS1_DONE, RS_GS2, RS_GIVENS };

struct KPtrs {
    double *partials, *red, *H, *cs, *sn, *g, *coef, *misc, *status;
    int *guard, *done;
};

// The single-lane step OP on the column sums in P.red (run by one lane of the last workgroup).
template <int OP>
__device__ __forceinline__ void step_tail(const KPtrs &P, int k, int m) {
    if constexpr (OP == RS_BETA_START_ZERO) {   // the solve's first reduction (one column): also
        beta_body(0, m, P.red, P.g, P.misc, P.status, ST_NUM);   // clears the completion count
        beta_body(0, m, P.red, nullptr, P.misc, P.status, ST_BETA);
        *P.done = 0;
    } else if constexpr (OP == RS_BETA_START_X) {
        beta_body(0, m, P.red, nullptr, P.misc, P.status, ST_NUM);
        *P.done = 0;
    } else if constexpr (OP == RS_BETA) {
        beta_body(0, m, P.red, P.g, P.misc, P.status, ST_BETA);
    } else if constexpr (OP == RS_GS1) {
        gs1_body(0, k, m, P.red, P.H, P.coef, P.misc);
    } else if constexpr (OP == RS_GS1_DONE) {
        gs1_done_body(0, P.red, P.misc, P.guard);
    } else if constexpr (OP == RS_GS2) {
        gs2_body(0, k, m, P.red, P.H, P.coef, P.guard);
    } else {
        givens_body(0, k, m, P.red, P.guard, P.H, P.cs, P.sn, P.g, P.misc, P.status);
    }
}

// k_reduce_cols followed by single-lane step OP on the column sums, in one launch: each
// workgroup reduces its column (or nothing when the guard says skip), then counts itself done;
// the last one (agent-scope fences on both sides of the count, so the other columns' sums are
// visible to it) runs the step and clears the count for the next launch. The step runs even when
// the reduction was skipped (the Givens step needs it either way; the guarded steps check the
// guard themselves).
template <int OP>
__global__ __launch_bounds__(WG) void k_reduce_step(KPtrs P, int nb, const int *guard, int k, int m) {
    reduce_cols_body(blockIdx.x, P.partials, nb, P.red, guard);
    __shared__ int last;
    if (threadIdx.x == 0) {
        int is_last = 1;
        if (gridDim.x > 1) {
            __threadfence();
            is_last = atomicAdd(P.done, 1) == (int)gridDim.x - 1;
            if (is_last) {
                __threadfence();
                *P.done = 0;
            }
        }
        last = is_last;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    step_tail<OP>(P, k, m);
}

// ---- small systems (at most FOLD_NB vector workgroups): the dot and update kernels reduce their
// own partials in their last workgroup and run the step there, one launch instead of two. The
// columns are summed by reduce_cols_body, in the same order, so the results are those of the
// two-launch form bit for bit.
constexpr int FOLD_NB = 64;

// true in the last workgroup to finish (every workgroup's partials then visible to all its
// lanes); clears the count for the next launch
__device__ __forceinline__ bool last_workgroup(int *done) {
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int is_last = 1;
        if (gridDim.x > 1) {
            is_last = atomicAdd(done, 1) == (int)gridDim.x - 1;
            if (is_last) *done = 0;
        }
        last = is_last;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

template <int OP>
__global__ __launch_bounds__(WG) void k_mdot_step(int64_t len, const double *__restrict__ V, int64_t ldv, int q,
                                                  const double *__restrict__ w, KPtrs P, int nb, const int *guard,
                                                  int k, int m) {
    mdot_body(blockIdx.x, len, V, ldv, q, w, P.partials, nb, guard);
    if (!last_workgroup(P.done)) return;
    for (int c = 0; c <= q; ++c) {
        reduce_cols_body(c, P.partials, nb, P.red, guard);
        __syncthreads();
    }
    if (threadIdx.x == 0) step_tail<OP>(P, k, m);
}

template <int OP>
__global__ __launch_bounds__(WG) void k_update_step(int64_t len, const double *__restrict__ V, int64_t ldv, int q,
                                                    const double *__restrict__ c, double alpha, double *__restrict__ w,
                                                    KPtrs P, int nb, const int *guard, int k, int m) {
    update_body(gridDim.x - 1 - blockIdx.x, len, V, ldv, q, c, alpha, w, P.partials, guard);
    if (!last_workgroup(P.done)) return;
    reduce_cols_body(0, P.partials, nb, P.red, guard);
    __syncthreads();
    if (threadIdx.x == 0) step_tail<OP>(P, k, m);
}

// v = w / h (h read from device memory; left unchanged if h == 0)
__global__ __launch_bounds__(WG) void k_scale(int64_t len, const double *w, double *v, const double *h) {
    scale_body(blockIdx.x, len, w, v, h);
}

// ---- single-lane steps on the small dense Hessenberg problem (column-major, ld = m+1). After the
// first Gram-Schmidt pass: H(0:k,k) = dots, coef = dots, nrm0 = ||w|| before (gs1). After the
// first update: a second pass (guard = 1) if ||w'|| < ||w|| / sqrt(2) (gs1_done). After the second
// dot pass, only if guard: H(0:k,k) += dots2, coef = dots2 (gs2). Final norm, Givens rotations,
// residual estimate (givens). All run fused into the reduction before them (k_reduce_step).

// Back substitution on the k x k upper triangle: coef = y.
__global__ void k_solve(int k, int m, const double *__restrict__ H, const double *__restrict__ g, double *coef) {
    solve_body(blockIdx.x, k, m, H, g, coef);
}

__global__ __launch_bounds__(WG) void k_zero(int64_t len, double *v) {
    zero_body(blockIdx.x, len, v);
}

// ---- ILU residual: sums of ||(LU - A)_ij||^2 and ||A_ij||^2 over the pattern (factor layout)
template <typename T>
__global__ __launch_bounds__(WG) void k_ilu_residual(int n, int ZL, const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ colidx,
                                                     const int32_t *__restrict__ diag_pos,
                                                     const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
                                                     const int32_t *__restrict__ pair_ptr,
                                                     const int32_t *__restrict__ sik, const int32_t *__restrict__ skj,
                                                     const double *__restrict__ A, const T *__restrict__ X,
                                                     double *__restrict__ partial, int nb) {
    __shared__ double shn[WG / 64], shd[WG / 64];
    const int r = threadIdx.x & 3;
    double num = 0.0, den = 0.0;
    for (int pass = 0; pass < VEC_TILE / 4 / ROWS_PER_WG; ++pass) {
        const int i = (blockIdx.x * (VEC_TILE / 4 / ROWS_PER_WG) + pass) * ROWS_PER_WG + (threadIdx.x >> 2);
        if (i < n) {
            const int b0 = rowptr[i], b1 = rowptr[i + 1], d = diag_pos[i];
            for (int e = b0; e < b1; ++e) {
                const int j = colidx[e];
                double x[4], P[4];
                load_row(X + (int64_t)split_pos(e, i, b0, d, lrow[i], urow[i], ZL, n) * BB, r, x);
                if (i > j) {
                    double u[4];
                    load_row(X + ((int64_t)ZL + j) * BB, r, u);
                    row_times_block(x, u, P);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) P[c] = x[c];
                }
                for (int q = pair_ptr[e]; q < pair_ptr[e + 1]; ++q) {
                    double l[4], u[4], t[4];
                    load_row(X + (int64_t)sik[q] * BB, r, l);
                    load_row(X + (int64_t)skj[q] * BB, r, u);
                    row_times_block(l, u, t);
#pragma unroll
                    for (int c = 0; c < 4; ++c) P[c] += t[c];
                }
                double a[4];
                load_row(A + (int64_t)e * BB, r, a);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    num += (P[c] - a[c]) * (P[c] - a[c]);
                    den += a[c] * a[c];
                }
            }
        }
    }
    num = wave_sum(num);
    den = wave_sum(den);
    if ((threadIdx.x & 63) == 0) {
        shn[threadIdx.x >> 6] = num;
        shd[threadIdx.x >> 6] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = (shn[0] + shn[1]) + (shn[2] + shn[3]);
        partial[nb + blockIdx.x] = (shd[0] + shd[1]) + (shd[2] + shd[3]);
    }
}

struct Ctx {
    const abilu_pattern *p;
    Workspace W;
    char *work;
    hipStream_t s;
    int64_t nv;
    double *partials, *H, *cs, *sn, *g, *coef, *misc, *status, *red, *V, *Zb;
    int *guard, *done;
    int m;
    KPtrs ptrs() const { return KPtrs{partials, red, H, cs, sn, g, coef, misc, status, guard, done}; }
};

#define CKL()                                                     \
    do {                                                          \
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;    \
    } while (0)

// Column sums of the partials into c.red (ncols columns), then single-lane step op.
abilu_status reduce_step(Ctx &c, int ncols, const int *guard, int op, int k) {
    const int nb = c.W.nb_vec;
    ProfScope ps("fgmres_reduce", c.s, 8.0 * ncols * nb);
    const KPtrs P = c.ptrs();
    switch (op) {
        case RS_BETA_START_ZERO: k_reduce_step<RS_BETA_START_ZERO><<<ncols, WG, 0, c.s>>>(P, nb, guard, k, c.m); break;
        case RS_BETA_START_X: k_reduce_step<RS_BETA_START_X><<<ncols, WG, 0, c.s>>>(P, nb, guard, k, c.m); break;
        case RS_BETA: k_reduce_step<RS_BETA><<<ncols, WG, 0, c.s>>>(P, nb, guard, k, c.m); break;
        case RS_GS1: k_reduce_step<RS_GS1><<<ncols, WG, 0, c.s>>>(P, nb, guard, k, c.m); break;
        case RS_GS1_DONE: k_reduce_step<RS_GS1_DONE><<<ncols, WG, 0, c.s>>>(P, nb, guard, k, c.m); break;
        case RS_GS2: k_reduce_step<RS_GS2><<<ncols, WG, 0, c.s>>>(P, nb, guard, k, c.m); break;
        default: k_reduce_step<RS_GIVENS><<<ncols, WG, 0, c.s>>>(P, nb, guard, k, c.m); break;
    }
    CKL();
    return ABILU_OK;
}

// one launch of kernel template K<OP> for a runtime op (the steps after a dot or update kernel)
#define ABILU_STEP_SWITCH(K, ARGS)                                                  \
    switch (op) {                                                                   \
        case RS_BETA: K<RS_BETA><<<nb, WG, 0, c.s>>> ARGS; break;                   \
        case RS_GS1: K<RS_GS1><<<nb, WG, 0, c.s>>> ARGS; break;                     \
        case RS_GS1_DONE: K<RS_GS1_DONE><<<nb, WG, 0, c.s>>> ARGS; break;           \
        case RS_GS2: K<RS_GS2><<<nb, WG, 0, c.s>>> ARGS; break;                     \
        default: K<RS_GIVENS><<<nb, WG, 0, c.s>>> ARGS; break;                      \
    }

// c.red[0..q] <- dots of w with V_0..V_{q-1}, then ||w||^2; then step op
abilu_status mdot_reduce(Ctx &c, const double *Vb, int q, const double *w, const int *guard, int op, int k) {
    const int nb = c.W.nb_vec;
    const double n8 = 8.0 * (double)c.nv;
    if (nb <= FOLD_NB && op != RS_BETA_START_ZERO && op != RS_BETA_START_X) {
        {
            ProfScope ps("fgmres_mdot", c.s, (q + 1) * n8 + 8.0 * (q + 1) * nb);
            const KPtrs P = c.ptrs();
            ABILU_STEP_SWITCH(k_mdot_step, (c.nv, Vb, c.nv, q, w, P, nb, guard, k, c.m))
        }
        CKL();
        return ABILU_OK;
    }
    {
        ProfScope ps("fgmres_mdot", c.s, (q + 1) * n8);
        k_mdot<<<nb, WG, 0, c.s>>>(c.nv, Vb, c.nv, q, w, c.partials, nb, guard);
    }
    CKL();
    return reduce_step(c, q + 1, guard, op, k);
}

// w += alpha * sum_k coef[k] Vb_k; with a step op (>= 0): c.red[0] <- ||w||^2 afterwards, then the step
abilu_status update_reduce(Ctx &c, const double *Vb, int q, double alpha, double *w, const int *guard, int op, int k) {
    const int nb = c.W.nb_vec;
    const double n8 = 8.0 * (double)c.nv;
    const bool with_norm = op >= 0;
    if (with_norm && nb <= FOLD_NB) {
        {
            ProfScope ps("fgmres_update", c.s, (q + 2) * n8 + 8.0 * nb);
            const KPtrs P = c.ptrs();
            ABILU_STEP_SWITCH(k_update_step, (c.nv, Vb, c.nv, q, c.coef, alpha, w, P, nb, guard, k, c.m))
        }
        CKL();
        return ABILU_OK;
    }
    {
        ProfScope ps("fgmres_update", c.s, (q + 2) * n8);
        k_update<<<nb, WG, 0, c.s>>>(c.nv, Vb, c.nv, q, c.coef, alpha, w, with_norm ? c.partials : nullptr, guard);
    }
    CKL();
    return with_norm ? reduce_step(c, 1, guard, op, k) : ABILU_OK;
}

// copies the flag word and the status scalars to the host
abilu_status readback(Ctx &c, double *h, uint32_t *flags) {
    if (!hip_ok(hipMemcpyAsync(c.p->pinned, c.work, 128, hipMemcpyDeviceToHost, c.s), "fgmres readback"))
        return ABILU_EDEVICE;
    if (!hip_ok(hipStreamSynchronize(c.s), "fgmres readback sync")) return ABILU_EDEVICE;
    *flags = *(const uint32_t *)c.p->pinned;
    for (int q = 0; q < 8; ++q) h[q] = c.p->pinned[8 + q];
    return ABILU_OK;
}

// r = b - A x into V_0, beta = ||r|| into g[0], misc[MI_BETA] and status[ST_BETA]. The SpMV runs
// its workgroups descending (measured slightly faster than ascending after either predecessor).
abilu_status true_residual(Ctx &c, const double *A, const double *b, const double *x) {
    abilu_status st = spmv_impl(c.p, A, x, c.V, b, true, c.s);
    if (st != ABILU_OK) return st;
    return mdot_reduce(c, c.V, 0, c.V, nullptr, RS_BETA, 0);
}

}  // namespace

extern "C" abilu_status fgmres_solve(const abilu_pattern *p, const double *d_A, const double *d_b, double *d_x,
                                     int32_t restart, int32_t maxit, double rtol, const void *d_LU,
                                     const void *d_Dinv, abilu_prec prec, int32_t apply_sweeps, abilu_mode mode,
                                     uint32_t options, void *d_work, size_t work_bytes, void *stream,
                                     abilu_fgmres_result *out) {
    if (!p || !out || !d_work) return ABILU_EINVAL;
    if (restart < 1 || restart > MAX_RESTART || maxit < 0 || !(rtol >= 0.0) || apply_sweeps < 0) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    if (!mode_ok(p, mode)) return ABILU_EINVAL;
    *out = abilu_fgmres_result{0, 0, 0, 0u, 0, 0.0, 0.0};
    Ctx c;
    c.p = p;
    c.W = layout(p, prec, restart);
    if (work_bytes < c.W.total) return ABILU_EINVAL;
    if (p->n == 0) {
        out->converged = 1;
        return ABILU_OK;
    }
    if (!d_A || !d_b || !d_x) return ABILU_EINVAL;
    if (apply_sweeps > 0 && (!d_LU || !d_Dinv)) return ABILU_EINVAL;
    c.work = (char *)d_work;
    c.s = (hipStream_t)stream;
    c.nv = 4 * (int64_t)p->n;
    const int m = restart;
    c.partials = (double *)(c.work + c.W.partials);
    c.H = (double *)(c.work + c.W.hess);
    c.cs = (double *)(c.work + c.W.cs);
    c.sn = (double *)(c.work + c.W.sn);
    c.g = (double *)(c.work + c.W.g);
    c.coef = (double *)(c.work + c.W.coef);
    c.misc = (double *)(c.work + c.W.misc);
    c.status = (double *)(c.work + c.W.status);
    c.red = (double *)(c.work + c.W.red);
    c.V = (double *)(c.work + c.W.V);
    c.Zb = (double *)(c.work + c.W.Z);
    c.guard = (int *)(c.misc + MI_GUARD);
    c.done = (int *)(c.misc + MI_DONE);
    c.m = m;
    double h[8];
    uint32_t flags = 0;
    abilu_status st;

    // ||b|| and the initial residual (b itself for a zero initial guess)
    const bool zero_guess = (options & ABILU_FGMRES_ZERO_GUESS) != 0;
    if ((st = mdot_reduce(c, c.V, 0, d_b, nullptr, zero_guess ? RS_BETA_START_ZERO : RS_BETA_START_X, 0)) !=
        ABILU_OK)
        return st;
    const double *first_v0 = c.V;   // the vector the first cycle normalises into V_0
    if (zero_guess) {
        {
            ProfScope ps("fgmres_scale", c.s, 8.0 * (double)c.nv);
            k_zero<<<c.W.nb_vec, WG, 0, c.s>>>(c.nv, d_x);
        }
        CKL();
        first_v0 = d_b;
    } else if ((st = true_residual(c, d_A, d_b, d_x)) != ABILU_OK) {
        return st;
    }
    if ((st = readback(c, h, &flags)) != ABILU_OK) return st;
    const double bnorm = h[ST_NUM];
    const double bn = bnorm > 0 ? bnorm : 1.0;
    const double tol = rtol * bn;
    double beta = h[ST_BETA], est = beta;
    int iters = 0, restarts = 0, reorth = 0;
    bool converged = beta <= tol;
    bool nonfinite = !std::isfinite(beta) || !std::isfinite(bnorm);

    while (!converged && !nonfinite && iters < maxit && beta > 0.0) {
        {
            ProfScope ps("fgmres_scale", c.s, 16.0 * (double)c.nv);
            k_scale<<<c.W.nb_vec, WG, 0, c.s>>>(c.nv, first_v0, c.V, c.misc + MI_BETA);
        }
        CKL();
        first_v0 = c.V;
        int k = 0;
        while (k < m && iters < maxit) {
            const double *vk = c.V + (int64_t)k * c.nv;
            double *zk = c.Zb + (int64_t)k * c.nv;
            double *w = c.V + (int64_t)(k + 1) * c.nv;
            if ((st = apply_impl(p, d_LU, d_Dinv, prec, vk, zk, apply_sweeps, mode, c.work, c.W, c.s)) != ABILU_OK)
                return st;
            if ((st = spmv_impl(p, d_A, zk, w, nullptr, !apply_ends_descending(apply_sweeps, mode), c.s)) !=
                ABILU_OK)
                return st;
            // Gram-Schmidt pass 1
            // pass 1: dots, H(0:k,k); update, then the decision on a second pass
            if ((st = mdot_reduce(c, c.V, k + 1, w, nullptr, RS_GS1, k)) != ABILU_OK) return st;
            if ((st = update_reduce(c, c.V, k + 1, -1.0, w, nullptr, RS_GS1_DONE, k)) != ABILU_OK) return st;
            // pass 2, executed by the device only when the guard is set; the Givens step after its
            // update runs either way
            const int pass2_begin = prof_mark();
            if ((st = mdot_reduce(c, c.V, k + 1, w, c.guard, RS_GS2, k)) != ABILU_OK) return st;
            if ((st = update_reduce(c, c.V, k + 1, -1.0, w, c.guard, RS_GIVENS, k)) != ABILU_OK) return st;
            const int pass2_end = prof_mark();
            {
                ProfScope ps("fgmres_scale", c.s, 16.0 * (double)c.nv);
                k_scale<<<c.W.nb_vec, WG, 0, c.s>>>(c.nv, w, w, c.misc + MI_HN);
            }
            CKL();
            if ((st = readback(c, h, &flags)) != ABILU_OK) return st;
            if (h[ST_GUARD] != 0.0)
                ++reorth;
            else
                prof_cancel_bytes(pass2_begin, pass2_end);   // the second pass exited at once
            ++iters;
            ++k;
            est = h[ST_EST];
            if (!std::isfinite(est) || !std::isfinite(h[ST_HN])) {
                nonfinite = true;
                break;
            }
            if (est <= tol || h[ST_HN] == 0.0) break;
        }
        if (nonfinite) break;
        // least squares and x += Z y
        {
            ProfScope ps("fgmres_small", c.s);
            k_solve<<<1, 1, 0, c.s>>>(k, m, c.H, c.g, c.coef);
        }
        CKL();
        if ((st = update_reduce(c, c.Zb, k, 1.0, d_x, nullptr, -1, 0)) != ABILU_OK) return st;
        if ((st = true_residual(c, d_A, d_b, d_x)) != ABILU_OK) return st;
        if ((st = readback(c, h, &flags)) != ABILU_OK) return st;
        ++restarts;
        beta = h[ST_BETA];
        if (!std::isfinite(beta)) nonfinite = true;
        converged = beta <= tol;
    }
    out->iters = iters;
    out->restarts = restarts;
    out->converged = converged ? 1 : 0;
    out->flags = flags;
    out->reorth = reorth;
    out->rel_true_residual = beta / bn;
    out->rel_estimate = est / bn;
    if (nonfinite) return ABILU_ENONFINITE;
    if (!converged) return ABILU_WARN_NOCONV;
    if (flags & ABILU_FLAG_MODIFIED) return ABILU_WARN_MODIFIED;
    return ABILU_OK;
}

template <typename T>
static abilu_status ilu_residual_t(const abilu_pattern *p, const double *A, const T *X, char *work,
                                   const Workspace &W, double *h_rel, hipStream_t s) {
    const int nb = W.nb_vec;
    double *partial = (double *)(work + W.partials);
    double *red = (double *)(work + W.red);
    {
        ProfScope ps("ilu_residual", s);
        k_ilu_residual<T><<<nb, WG, 0, s>>>(p->n, (int)p->nnzb_lower, p->rowptr, p->colidx, p->diag_pos, p->lrow,
                                            p->urow, p->pair_ptr, p->sik, p->skj, A, X, partial, nb);
    }
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    k_reduce_cols<<<2, WG, 0, s>>>(partial, nb, red, nullptr);
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    double v[2];
    if (!hip_ok(hipMemcpyAsync(p->pinned, red, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "residual readback"))
        return ABILU_EDEVICE;
    if (!hip_ok(hipStreamSynchronize(s), "residual readback sync")) return ABILU_EDEVICE;
    v[0] = p->pinned[0];
    v[1] = p->pinned[1];
    *h_rel = v[1] > 0 ? std::sqrt(v[0] / v[1]) : std::sqrt(v[0]);
    return ABILU_OK;
}

extern "C" abilu_status abilu_ilu_residual(const abilu_pattern *p, const double *d_A, const void *d_LU,
                                           abilu_prec prec, void *d_work, size_t work_bytes, double *h_rel,
                                           void *stream) {
    if (!p || !h_rel || !d_work) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    const Workspace W = layout(p, prec, 0);
    if (work_bytes < W.total) return ABILU_EINVAL;
    if (p->n == 0) {
        *h_rel = 0.0;
        return ABILU_OK;
    }
    if (!d_A || !d_LU) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (prec == ABILU_F32) return ilu_residual_t<float>(p, d_A, (const float *)d_LU, (char *)d_work, W, h_rel, s);
    return ilu_residual_t<double>(p, d_A, (const double *)d_LU, (char *)d_work, W, h_rel, s);
}
