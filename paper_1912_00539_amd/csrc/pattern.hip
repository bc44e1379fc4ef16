// Pattern analysis on the device: validation, diagonal positions and the update sets
// K(i,j) = { k < min(i,j) : (i,k), (k,j) in S_B } of the block ILU(0) equations (Section 4.2,
// equation bilu), stored as CSR lists of block-position pairs ascending in k.
#include <climits>
#include <cstring>

#include "abilu_internal.h"

namespace {

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

__global__ void k_pat_rows(int n, int64_t Z, const int32_t *__restrict__ rowptr,
                           const int32_t *__restrict__ colidx, int32_t *__restrict__ diag_pos,
                           unsigned *__restrict__ err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
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

// one thread per block row; counts |K(i,j)| for every block of the row
__global__ void k_pat_count(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                            int64_t *__restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b0 = rowptr[i], b1 = rowptr[i + 1];
    for (int e = b0; e < b1; ++e) {
        int j = colidx[e];
        int lim = i < j ? i : j;
        int c = 0;
        for (int f = b0; f < b1; ++f) {
            int k = colidx[f];
            if (k >= lim) break;
            c += (find_col(rowptr, colidx, k, j) >= 0);
        }
        cnt[e] = c;
    }
}

__global__ void k_pat_fill(int n, int ZL, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                           const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow,
                           const int32_t *__restrict__ urow, const int64_t *__restrict__ ptr,
                           int32_t *__restrict__ pik, int32_t *__restrict__ pkj, int32_t *__restrict__ sik,
                           int32_t *__restrict__ skj) {
    using abilu_dev::split_pos;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b0 = rowptr[i], b1 = rowptr[i + 1];
    for (int e = b0; e < b1; ++e) {
        int j = colidx[e];
        int lim = i < j ? i : j;
        int64_t o = ptr[e];
        for (int f = b0; f < b1; ++f) {
            int k = colidx[f];
            if (k >= lim) break;
            int g = find_col(rowptr, colidx, k, j);
            if (g >= 0) {
                pik[o] = f;
                pkj[o] = g;
                sik[o] = split_pos(f, i, b0, diag_pos[i], lrow[i], urow[i], ZL, n);
                skj[o] = split_pos(g, k, rowptr[k], diag_pos[k], lrow[k], urow[k], ZL, n);
                ++o;
            }
        }
    }
}

// per-row counts of strictly lower / upper blocks
__global__ void k_pat_tri_counts(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ diag_pos,
                                 int64_t *__restrict__ nl, int64_t *__restrict__ nu) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    nl[i] = diag_pos[i] - rowptr[i];
    nu[i] = rowptr[i + 1] - diag_pos[i] - 1;
}

// columns of the lower and upper parts in factor-layout order
__global__ void k_pat_tri_cols(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                               const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow,
                               const int32_t *__restrict__ urow, int32_t *__restrict__ lcol,
                               int32_t *__restrict__ ucol) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b0 = rowptr[i], d = diag_pos[i], b1 = rowptr[i + 1];
    for (int e = b0; e < d; ++e) lcol[lrow[i] + (e - b0)] = colidx[e];
    for (int e = d + 1; e < b1; ++e) ucol[urow[i] + (e - d - 1)] = colidx[e];
}

void free_pattern(abilu_pattern *p) {
    if (!p) return;
    (void)hipFree(p->rowptr);
    (void)hipFree(p->colidx);
    (void)hipFree(p->diag_pos);
    (void)hipFree(p->pair_ptr);
    (void)hipFree(p->pik);
    (void)hipFree(p->pkj);
    (void)hipFree(p->sik);
    (void)hipFree(p->skj);
    (void)hipFree(p->lrow);
    (void)hipFree(p->urow);
    (void)hipFree(p->lcol);
    (void)hipFree(p->ucol);
    if (p->pinned) (void)hipHostFree(p->pinned);
    delete p;
}

}  // namespace

extern "C" abilu_status abilu_build_pattern(int32_t nbrows, const int32_t *d_rowptr,
                                            const int32_t *d_colidx, int32_t bs, void *stream,
                                            abilu_pattern **out) {
    using namespace abilu;
    if (!out) return ABILU_EINVAL;
    *out = nullptr;
    if (bs != 4 || nbrows < 0 || !d_rowptr) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = nbrows;

    abilu_pattern *p = new abilu_pattern();
    int64_t *cnt = nullptr, *scan = nullptr, *tot = nullptr, *ptr64 = nullptr;
    unsigned *err = nullptr;
    abilu_status st = ABILU_OK;
    int32_t ends[2] = {0, 0};
#define CK(x)                                  \
    do {                                       \
        if (!hip_ok((x), #x)) {                \
            st = ABILU_EDEVICE;                \
            goto fail;                         \
        }                                      \
    } while (0)
#define CKA(x)                                 \
    do {                                       \
        if (!hip_ok((x), #x)) {                \
            st = ABILU_ENOMEM;                 \
            goto fail;                         \
        }                                      \
    } while (0)
    {
        CK(hipGetDevice(&p->device));
        p->n = n;
        CK(hipMemcpyAsync(&ends[0], d_rowptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(&ends[1], d_rowptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        if (ends[0] != 0 || ends[1] < n) { st = ABILU_EPATTERN; goto fail; }
        const int64_t Z = ends[1];
        if (Z > 0 && !d_colidx) { st = ABILU_EINVAL; goto fail; }
        p->nnzb = Z;
        CKA(hipHostMalloc((void **)&p->pinned, 64 * sizeof(double), hipHostMallocDefault));
        CKA(hipMalloc(&p->rowptr, sizeof(int32_t) * (n + 1)));
        CKA(hipMalloc(&p->colidx, sizeof(int32_t) * (Z + 1)));
        CKA(hipMalloc(&p->diag_pos, sizeof(int32_t) * (n + 1)));
        CKA(hipMalloc(&p->pair_ptr, sizeof(int32_t) * (Z + 1)));
        CKA(hipMalloc(&err, sizeof(unsigned)));
        CK(hipMemcpyAsync(p->rowptr, d_rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
        if (Z > 0) CK(hipMemcpyAsync(p->colidx, d_colidx, sizeof(int32_t) * Z, hipMemcpyDeviceToDevice, s));
        CK(hipMemsetAsync(err, 0, sizeof(unsigned), s));
        if (n > 0) {
            k_pat_rows<<<div_up(n, 256), 256, 0, s>>>(n, Z, p->rowptr, p->colidx, p->diag_pos, err);
            CK(hipGetLastError());
        }
        unsigned herr = 0;
        CK(hipMemcpyAsync(&herr, err, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        if (herr) { st = ABILU_EPATTERN; goto fail; }
        const int ntmax = scan_tiles(Z > n ? Z : n);
        CKA(hipMalloc(&cnt, sizeof(int64_t) * (Z + n + 2)));
        CKA(hipMalloc(&scan, sizeof(int64_t) * (Z + n + 2)));
        CKA(hipMalloc(&ptr64, sizeof(int64_t) * (Z + n + 2)));
        CKA(hipMalloc(&tot, sizeof(int64_t) * (ntmax + 1)));
        CKA(hipMalloc(&p->lrow, sizeof(int32_t) * (n + 1)));
        CKA(hipMalloc(&p->urow, sizeof(int32_t) * (n + 1)));
        // row offsets of the strictly lower / upper parts of the factor layout
        int64_t tri[2] = {0, 0};
        if (n > 0) {
            k_pat_tri_counts<<<div_up(n, 256), 256, 0, s>>>(n, p->rowptr, p->diag_pos, cnt, cnt + (n + 1));
            CK(hipGetLastError());
        }
        for (int part = 0; part < 2; ++part) {
            const int64_t *counts = cnt + (part == 0 ? 0 : (n + 1));
            CK(scan_exclusive(n, counts, scan, tot, ptr64, part == 0 ? p->lrow : p->urow, s));
            CK(hipMemcpyAsync(&tri[part], ptr64 + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            CK(hipStreamSynchronize(s));
        }
        p->nnzb_lower = tri[0];
        p->nnzb_upper = tri[1];
        if (tri[0] + tri[1] + n != Z) { st = ABILU_EPATTERN; goto fail; }
        CKA(hipMalloc(&p->lcol, sizeof(int32_t) * (tri[0] + 1)));
        CKA(hipMalloc(&p->ucol, sizeof(int32_t) * (tri[1] + 1)));
        CK(hipMemsetAsync(p->lcol, 0, sizeof(int32_t) * (tri[0] + 1), s));
        CK(hipMemsetAsync(p->ucol, 0, sizeof(int32_t) * (tri[1] + 1), s));
        if (n > 0) {
            k_pat_tri_cols<<<div_up(n, 256), 256, 0, s>>>(n, p->rowptr, p->colidx, p->diag_pos, p->lrow, p->urow,
                                                           p->lcol, p->ucol);
            CK(hipGetLastError());
        }

        // update sets: counts, offsets, lists (CSR positions and factor-layout positions)
        if (n > 0) {
            k_pat_count<<<div_up(n, 128), 128, 0, s>>>(n, p->rowptr, p->colidx, cnt);
            CK(hipGetLastError());
        }
        CK(scan_exclusive(Z, cnt, scan, tot, ptr64, p->pair_ptr, s));
        int64_t npairs = 0;
        CK(hipMemcpyAsync(&npairs, ptr64 + Z, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        if (npairs < 0 || npairs > (int64_t)INT_MAX) { st = ABILU_EPATTERN; goto fail; }
        p->npairs = npairs;
        CKA(hipMalloc(&p->pik, sizeof(int32_t) * (npairs + 1)));
        CKA(hipMalloc(&p->pkj, sizeof(int32_t) * (npairs + 1)));
        CKA(hipMalloc(&p->sik, sizeof(int32_t) * (npairs + 1)));
        CKA(hipMalloc(&p->skj, sizeof(int32_t) * (npairs + 1)));
        if (n > 0 && npairs > 0) {
            k_pat_fill<<<div_up(n, 128), 128, 0, s>>>(n, (int)tri[0], p->rowptr, p->colidx, p->diag_pos, p->lrow,
                                                       p->urow, ptr64, p->pik, p->pkj, p->sik, p->skj);
            CK(hipGetLastError());
        }
        CK(hipStreamSynchronize(s));
    }
    (void)hipFree(cnt);
    (void)hipFree(scan);
    (void)hipFree(ptr64);
    (void)hipFree(tot);
    (void)hipFree(err);
    *out = p;
    return ABILU_OK;
fail:
    (void)hipStreamSynchronize(s);
    (void)hipFree(cnt);
    (void)hipFree(scan);
    (void)hipFree(ptr64);
    (void)hipFree(tot);
    (void)hipFree(err);
    free_pattern(p);
    return st;
#undef CK
#undef CKA
}

extern "C" abilu_status abilu_pattern_destroy(abilu_pattern *p) {
    free_pattern(p);
    return ABILU_OK;
}

extern "C" abilu_status abilu_pattern_info(const abilu_pattern *p, int32_t *nbrows, int64_t *nnzb,
                                           int64_t *npairs) {
    if (!p) return ABILU_EINVAL;
    if (nbrows) *nbrows = p->n;
    if (nnzb) *nnzb = p->nnzb;
    if (npairs) *npairs = p->npairs;
    return ABILU_OK;
}

extern "C" abilu_status abilu_pattern_export(const abilu_pattern *p, int32_t *d_diag_pos,
                                             int32_t *d_pair_ptr, int32_t *d_pik, int32_t *d_pkj,
                                             void *stream) {
    if (!p) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (d_diag_pos && p->n > 0)
        e = hipMemcpyAsync(d_diag_pos, p->diag_pos, sizeof(int32_t) * p->n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_pair_ptr)
        e = hipMemcpyAsync(d_pair_ptr, p->pair_ptr, sizeof(int32_t) * (p->nnzb + 1), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_pik && p->npairs > 0)
        e = hipMemcpyAsync(d_pik, p->pik, sizeof(int32_t) * p->npairs, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_pkj && p->npairs > 0)
        e = hipMemcpyAsync(d_pkj, p->pkj, sizeof(int32_t) * p->npairs, hipMemcpyDeviceToDevice, s);
    return abilu::hip_ok(e, "pattern export copy") ? ABILU_OK : ABILU_EDEVICE;
}
