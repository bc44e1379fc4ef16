// Diagnostics of a factor (Section 6.2): the largest entry-wise difference between two factors,
// split into the strictly lower part (L) and the diagonal and strictly upper part (U) -- numerator
// and denominator of the factor errors ||vec(L - L_ilu)||_inf / ||vec(L_0 - L_ilu)||_inf and
// likewise for U -- and the max-norms of the Jacobi iteration matrices of the two triangular solves,
// ||L_strict||_inf and ||U_diag^{-1} U_strict||_inf (largest absolute scalar row sum).
//
// Both reduce through per-workgroup partials (workspace) and one small max kernel. The max keeps a
// NaN if one occurs, so a non-finite factor shows in the result.
#include "kernels.h"

using namespace abilu;
using namespace abilu_dev;
using namespace abilu_k;

namespace {

// max that keeps NaN (of either operand)
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Writes the workgroup's maxima of a and b to partial[blk] and partial[nb + blk].
__device__ __forceinline__ void block_max2(double a, double b, double *partial, int nb) {
    __shared__ double sa[WG / 64], sb[WG / 64];
    a = wave_max(a);
    b = wave_max(b);
    if ((threadIdx.x & 63) == 0) {
        sa[threadIdx.x >> 6] = a;
        sb[threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = nanmax(nanmax(sa[0], sa[1]), nanmax(sa[2], sa[3]));
        partial[nb + blockIdx.x] = nanmax(nanmax(sb[0], sb[1]), nanmax(sb[2], sb[3]));
    }
}

// max |X - Y| over the first nl entries (strictly lower blocks) and over the rest, grid-stride.
template <typename T>
__global__ __launch_bounds__(WG) void k_factor_maxdiff(int64_t len, int64_t nl, const T *__restrict__ X,
                                                       const double *__restrict__ Y, double *__restrict__ partial,
                                                       int nb) {
    double ml = 0.0, mu = 0.0;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x; t < len; t += stride) {
        const double d = fabs((double)X[t] - Y[t]);
        if (t < nl) ml = nanmax(ml, d);
        else mu = nanmax(mu, d);
    }
    block_max2(ml, mu, partial, nb);
}

// Row sums of |L_ij| (j < i) and of |(Dinv_i U_ij)| (j > i) for every scalar row; one quad per
// block row, lane r on scalar row r, rows grid-stride. Block products in the factor precision,
// sums in double, blocks in ascending column order.
template <typename T>
__global__ __launch_bounds__(WG) void k_jacobi_norms(int n, const int32_t *__restrict__ lrow,
                                                     const int32_t *__restrict__ urow, const T *__restrict__ Lb,
                                                     const T *__restrict__ Ub, const T *__restrict__ Dinv,
                                                     double *__restrict__ partial, int nb) {
    const int r = threadIdx.x & 3;
    double ml = 0.0, mu = 0.0;
    for (int i = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2); i < n; i += gridDim.x * ROWS_PER_WG) {
        double sl = 0.0, su = 0.0;
        for (int e = lrow[i]; e < lrow[i + 1]; ++e) {
            T l[4];
            load_row(Lb + (int64_t)e * BB, r, l);
#pragma unroll
            for (int c = 0; c < 4; ++c) sl += fabs((double)l[c]);
        }
        T dr[4];
        load_row(Dinv + (int64_t)i * BB, r, dr);
        for (int e = urow[i]; e < urow[i + 1]; ++e) {
            T u[4], P[4];
            load_row(Ub + (int64_t)e * BB, r, u);
            row_times_block(dr, u, P);
#pragma unroll
            for (int c = 0; c < 4; ++c) su += fabs((double)P[c]);
        }
        ml = nanmax(ml, sl);
        mu = nanmax(mu, su);
    }
    block_max2(ml, mu, partial, nb);
}

// out[c] = max over partial[c * nb .. c * nb + nb), one workgroup per column
__global__ __launch_bounds__(WG) void k_max_cols(const double *__restrict__ partial, int nb, double *__restrict__ out) {
    __shared__ double sh[WG / 64];
    const double *pc = partial + (int64_t)blockIdx.x * nb;
    double m = 0.0;
    for (int b = threadIdx.x; b < nb; b += WG) m = nanmax(m, pc[b]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = nanmax(nanmax(sh[0], sh[1]), nanmax(sh[2], sh[3]));
}

// reduce the two partial columns and read them back (blocks on s)
abilu_status finish_max2(const abilu_pattern *p, double *partial, int nb, double *red, double *h_a, double *h_b,
                         hipStream_t s) {
    k_max_cols<<<2, WG, 0, s>>>(partial, nb, red);
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    if (!hip_ok(hipMemcpyAsync(p->pinned, red, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "diagnostic readback"))
        return ABILU_EDEVICE;
    if (!hip_ok(hipStreamSynchronize(s), "diagnostic readback sync")) return ABILU_EDEVICE;
    *h_a = p->pinned[0];
    *h_b = p->pinned[1];
    return ABILU_OK;
}

// The diagnostics' scratch: 2 nb partial maxima, then 2 results, from byte 256 of the workspace
// (the region after the header, which every workspace of either precision has room for: it holds
// at least the factor ping-pong buffers and the reduction areas). Returns false when too small.
struct DiagScratch {
    double *partial, *red;
    int nb;
};
bool diag_scratch(const abilu_pattern *p, void *work, size_t work_bytes, DiagScratch *out) {
    const Workspace W = layout(p, ABILU_F32, 0);    // the smaller of the two precisions' layouts
    if (work_bytes < W.total) return false;
    const size_t part = ((size_t)16 * W.nb_vec + 255) & ~(size_t)255;
    if (256 + part + 256 > W.total) return false;
    out->nb = W.nb_vec;
    out->partial = (double *)((char *)work + 256);
    out->red = (double *)((char *)work + 256 + part);
    return true;
}

template <typename T>
abilu_status maxdiff_t(const abilu_pattern *p, const T *X, const double *Y, const DiagScratch &D, double *h_lower,
                       double *h_upper, hipStream_t s) {
    {
        ProfScope ps("factor_maxdiff", s, (sizeof(T) + 8.0) * 16.0 * (double)p->nnzb);
        k_factor_maxdiff<T><<<D.nb, WG, 0, s>>>(16 * p->nnzb, 16 * p->nnzb_lower, X, Y, D.partial, D.nb);
    }
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    return finish_max2(p, D.partial, D.nb, D.red, h_lower, h_upper, s);
}

template <typename T>
abilu_status jacobi_t(const abilu_pattern *p, const T *LU, const T *Dinv, const DiagScratch &D, double *h_l,
                      double *h_u, hipStream_t s) {
    const T *Ub = LU + ((int64_t)p->nnzb_lower + p->n) * BB;
    {
        ProfScope ps("jacobi_norms", s);
        k_jacobi_norms<T><<<D.nb, WG, 0, s>>>(p->n, p->lrow, p->urow, LU, Ub, Dinv, D.partial, D.nb);
    }
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    return finish_max2(p, D.partial, D.nb, D.red, h_l, h_u, s);
}

}  // namespace

extern "C" abilu_status abilu_factor_maxdiff(const abilu_pattern *p, abilu_prec prec, const void *d_X,
                                             const double *d_Y, void *d_work, size_t work_bytes, double *h_lower,
                                             double *h_upper, void *stream) {
    if (!p || !d_work || !h_lower || !h_upper) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    DiagScratch D;
    if (!diag_scratch(p, d_work, work_bytes, &D)) return ABILU_EINVAL;
    if (p->n == 0) {
        *h_lower = *h_upper = 0.0;
        return ABILU_OK;
    }
    if (!d_X || !d_Y) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (prec == ABILU_F32) return maxdiff_t<float>(p, (const float *)d_X, d_Y, D, h_lower, h_upper, s);
    return maxdiff_t<double>(p, (const double *)d_X, d_Y, D, h_lower, h_upper, s);
}

extern "C" abilu_status abilu_jacobi_norms(const abilu_pattern *p, abilu_prec prec, const void *d_LU,
                                           const void *d_Dinv, void *d_work, size_t work_bytes, double *h_norm_l,
                                           double *h_norm_u, void *stream) {
    if (!p || !d_work || !h_norm_l || !h_norm_u) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    DiagScratch D;
    if (!diag_scratch(p, d_work, work_bytes, &D)) return ABILU_EINVAL;
    if (p->n == 0) {
        *h_norm_l = *h_norm_u = 0.0;
        return ABILU_OK;
    }
    if (!d_LU || !d_Dinv) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (prec == ABILU_F32) return jacobi_t<float>(p, (const float *)d_LU, (const float *)d_Dinv, D, h_norm_l, h_norm_u, s);
    return jacobi_t<double>(p, (const double *)d_LU, (const double *)d_Dinv, D, h_norm_l, h_norm_u, s);
}
