// Pattern analysis on the device: validation, diagonal positions and the update sets
// K(i,j) = { k < min(i,j) : (i,k), (k,j) in S_B } of the block ILU(0) equations (Section 4.2,
// equation bilu), stored as CSR lists of block-position pairs ascending in k.
#include <climits>
#include <cstring>

#include "setup_kernels.h"

namespace {

using namespace abilu_setup;

__global__ void k_pat_rows(int n, int64_t Z, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                           int32_t *__restrict__ diag_pos, unsigned *__restrict__ err) {
    pat_rows_body(blockIdx.x, n, Z, rowptr, colidx, diag_pos, err);
}

__global__ __launch_bounds__(PAT_ROWS) void k_pat_count(int n, const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ colidx,
                                                         const int32_t *__restrict__ diag_pos,
                                                         int64_t *__restrict__ cnt) {
    pat_count_body(blockIdx.x, n, rowptr, colidx, diag_pos, cnt);
}

__global__ __launch_bounds__(PAT_ROWS) void k_pat_fill(int n, int ZL, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                           const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow,
                           const int32_t *__restrict__ urow, const int64_t *__restrict__ ptr,
                           int32_t *__restrict__ pik, int32_t *__restrict__ pkj, int32_t *__restrict__ sik,
                           int32_t *__restrict__ skj) {
    pat_fill_body(blockIdx.x, n, ZL, rowptr, colidx, diag_pos, lrow, urow, ptr, pik, pkj, sik, skj);
}

__global__ void k_pat_tri_counts(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ diag_pos,
                                 int64_t *__restrict__ nl, int64_t *__restrict__ nu) {
    pat_tri_counts_body(blockIdx.x, n, rowptr, diag_pos, nl, nu);
}

__global__ void k_pat_tri_cols(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                               const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ lrow,
                               const int32_t *__restrict__ urow, int32_t *__restrict__ lcol,
                               int32_t *__restrict__ ucol) {
    pat_tri_cols_body(blockIdx.x, n, rowptr, colidx, diag_pos, lrow, urow, lcol, ucol);
}

__global__ void k_pat_sym(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                          unsigned *__restrict__ asym) {
    pat_sym_body(blockIdx.x, n, rowptr, colidx, asym);
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
    abilu::free_chunks(p);
    if (p->pinned) (void)hipHostFree(p->pinned);
    delete p;
}

}  // namespace

namespace abilu {

size_t pattern_scratch_bytes(int32_t n, int64_t Z) {
    const int64_t len = Z + n + 2;
    return 256 + sizeof(int64_t) * (size_t)(2 * len + scan_tiles(Z > n ? Z : n) + 1);
}

// Non-blocking stage 1a: validation and diagonal positions; the error word (nonzero: invalid
// pattern) is copied to h_err when the stream reaches it.
abilu_status pattern_validate_async(int32_t n, int64_t Z, const int32_t *rowptr, const int32_t *colidx,
                                    int32_t *diag_pos, void *scratch, unsigned *h_err, hipStream_t s) {
    unsigned *err = (unsigned *)scratch;
    if (!hip_ok(hipMemsetAsync(err, 0, sizeof(unsigned), s), "pattern error clear")) return ABILU_EDEVICE;
    if (n > 0) {
        k_pat_rows<<<div_up(n, 256), 256, 0, s>>>(n, Z, rowptr, colidx, diag_pos, err);
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    }
    if (!hip_ok(hipMemcpyAsync(h_err, err, sizeof(unsigned), hipMemcpyDeviceToHost, s), "pattern error readback"))
        return ABILU_EDEVICE;
    return ABILU_OK;
}

// Non-blocking stage 1b (valid patterns only): lower/upper row offsets and the update-set
// offsets (pair_ptr); h_sizes receives ZL, ZU and the number of pairs. ptr64 in the scratch
// keeps the int64 pair offsets for pattern_fill.
abilu_status pattern_count_async(int32_t n, int64_t Z, const int32_t *rowptr, const int32_t *colidx,
                                 const int32_t *diag_pos, int32_t *lrow, int32_t *urow, int32_t *pair_ptr,
                                 void *scratch, int64_t *h_sizes, hipStream_t s) {
    const PatScratch S = pat_scratch(scratch, n, Z);
    int64_t *cnt = S.cnt, *ptr64 = S.ptr64, *tot = S.tot;
#define CK(x)                                              \
    do {                                                   \
        if (!hip_ok((x), #x)) return ABILU_EDEVICE;        \
    } while (0)
    if (n > 0) {
        k_pat_tri_counts<<<div_up(n, 256), 256, 0, s>>>(n, rowptr, diag_pos, cnt, cnt + (n + 1));
        CK(hipGetLastError());
    }
    for (int part = 0; part < 2; ++part) {
        CK(scan_exclusive(n, cnt + (part == 0 ? 0 : (n + 1)), tot, ptr64, part == 0 ? lrow : urow, s));
        CK(hipMemcpyAsync(h_sizes + part, ptr64 + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    if (n > 0) {
        k_pat_count<<<div_up(n, PAT_ROWS), PAT_ROWS, 0, s>>>(n, rowptr, colidx, diag_pos, cnt);
        CK(hipGetLastError());
    }
    CK(scan_exclusive(Z, cnt, tot, ptr64, pair_ptr, s));
    CK(hipMemcpyAsync(h_sizes + 2, ptr64 + Z, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    return ABILU_OK;
#undef CK
}

bool pattern_sizes_ok(int32_t n, int64_t Z, const int64_t *sizes) {
    return sizes[0] >= 0 && sizes[1] >= 0 && sizes[0] + sizes[1] + n == Z && sizes[2] >= 0 &&
           sizes[2] <= (int64_t)INT_MAX;
}

// Blocking stage 1 (two stream syncs).
abilu_status pattern_count(int32_t n, int64_t Z, const int32_t *rowptr, const int32_t *colidx, int32_t *diag_pos,
                           int32_t *lrow, int32_t *urow, int32_t *pair_ptr, void *scratch, int64_t *h_pinned,
                           hipStream_t s, int64_t *ZL, int64_t *ZU, int64_t *npairs) {
    abilu_status st = pattern_validate_async(n, Z, rowptr, colidx, diag_pos, scratch, (unsigned *)h_pinned, s);
    if (st != ABILU_OK) return st;
    if (!hip_ok(hipStreamSynchronize(s), "pattern validation sync")) return ABILU_EDEVICE;
    if (*(const unsigned *)h_pinned) return ABILU_EPATTERN;
    st = pattern_count_async(n, Z, rowptr, colidx, diag_pos, lrow, urow, pair_ptr, scratch, h_pinned, s);
    if (st != ABILU_OK) return st;
    if (!hip_ok(hipStreamSynchronize(s), "pattern count sync")) return ABILU_EDEVICE;
    *ZL = h_pinned[0];
    *ZU = h_pinned[1];
    *npairs = h_pinned[2];
    return pattern_sizes_ok(n, Z, h_pinned) ? ABILU_OK : ABILU_EPATTERN;
}

// Columns of the lower/upper parts and the update-set lists (non-blocking; the scratch must
// still hold what pattern_count left there).
abilu_status pattern_fill(int32_t n, int64_t Z, int64_t ZL, int64_t ZU, int64_t npairs, const int32_t *rowptr,
                          const int32_t *colidx, const int32_t *diag_pos, const int32_t *lrow, const int32_t *urow,
                          int32_t *lcol, int32_t *ucol, int32_t *pik, int32_t *pkj, int32_t *sik, int32_t *skj,
                          const void *scratch, hipStream_t s) {
    const int64_t *ptr64 = pat_scratch(const_cast<void *>(scratch), n, Z).ptr64;
    if (!hip_ok(hipMemsetAsync(lcol, 0, sizeof(int32_t) * (ZL + 1), s), "lcol clear") ||
        !hip_ok(hipMemsetAsync(ucol, 0, sizeof(int32_t) * (ZU + 1), s), "ucol clear"))
        return ABILU_EDEVICE;
    if (n > 0) {
        k_pat_tri_cols<<<div_up(n, 256), 256, 0, s>>>(n, rowptr, colidx, diag_pos, lrow, urow, lcol, ucol);
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    }
    if (n > 0 && npairs > 0) {
        k_pat_fill<<<div_up(n, PAT_ROWS), PAT_ROWS, 0, s>>>(n, (int)ZL, rowptr, colidx, diag_pos, lrow, urow, ptr64, pik, pkj,
                                                   sik, skj);
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    }
    return ABILU_OK;
}

}  // namespace abilu

extern "C" abilu_status abilu_build_pattern(int32_t nbrows, const int32_t *d_rowptr,
                                            const int32_t *d_colidx, int32_t bs, void *stream,
                                            abilu_pattern **out) {
    using namespace abilu;
    if (!out) return ABILU_EINVAL;
    *out = nullptr;
    if (bs != 4 || nbrows < 0 || nbrows == INT32_MAX || !d_rowptr) return ABILU_EINVAL;   // N + 1 fits int32
    hipStream_t s = (hipStream_t)stream;
    const int n = nbrows;

    abilu_pattern *p = new abilu_pattern();
    void *scratch = nullptr;
    abilu_status st = ABILU_OK;
    int32_t ends[2] = {0, 0};
    int64_t ZL = 0, ZU = 0, npairs = 0;
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
        CKA(hipMalloc(&p->lrow, sizeof(int32_t) * (n + 1)));
        CKA(hipMalloc(&p->urow, sizeof(int32_t) * (n + 1)));
        CKA(hipMalloc(&scratch, pattern_scratch_bytes(n, Z)));
        CK(hipMemcpyAsync(p->rowptr, d_rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
        if (Z > 0) CK(hipMemcpyAsync(p->colidx, d_colidx, sizeof(int32_t) * Z, hipMemcpyDeviceToDevice, s));
        st = pattern_count(n, Z, p->rowptr, p->colidx, p->diag_pos, p->lrow, p->urow, p->pair_ptr, scratch,
                           (int64_t *)p->pinned, s, &ZL, &ZU, &npairs);
        if (st != ABILU_OK) goto fail;
        p->nnzb_lower = ZL;
        p->nnzb_upper = ZU;
        p->npairs = npairs;
        CKA(hipMalloc(&p->lcol, sizeof(int32_t) * (ZL + 1)));
        CKA(hipMalloc(&p->ucol, sizeof(int32_t) * (ZU + 1)));
        CKA(hipMalloc(&p->pik, sizeof(int32_t) * (npairs + 1)));
        CKA(hipMalloc(&p->pkj, sizeof(int32_t) * (npairs + 1)));
        CKA(hipMalloc(&p->sik, sizeof(int32_t) * (npairs + 1)));
        CKA(hipMalloc(&p->skj, sizeof(int32_t) * (npairs + 1)));
        st = pattern_fill(n, Z, ZL, ZU, npairs, p->rowptr, p->colidx, p->diag_pos, p->lrow, p->urow, p->lcol,
                          p->ucol, p->pik, p->pkj, p->sik, p->skj, scratch, s);
        if (st != ABILU_OK) goto fail;
        // structural symmetry (the first factor sweep from A uses it to find the rows whose initial
        // inverse no other row forms)
        {
            unsigned *asym = (unsigned *)scratch;
            CK(hipMemsetAsync(asym, 0, sizeof(unsigned), s));
            if (n > 0) {
                k_pat_sym<<<div_up(n, 256), 256, 0, s>>>(n, p->rowptr, p->colidx, asym);
                CK(hipGetLastError());
            }
            CK(hipMemcpyAsync(p->pinned, asym, sizeof(unsigned), hipMemcpyDeviceToHost, s));
            CK(hipStreamSynchronize(s));
            p->symmetric = *(const unsigned *)p->pinned == 0;
        }
    }
    (void)hipFree(scratch);
    *out = p;
    return ABILU_OK;
fail:
    (void)hipStreamSynchronize(s);
    (void)hipFree(scratch);
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
                                           int64_t *npairs, int32_t *depth_D, int32_t *levels_lower,
                                           int32_t *levels_upper) {
    if (!p) return ABILU_EINVAL;
    if (nbrows) *nbrows = p->n;
    if (nnzb) *nnzb = p->nnzb;
    if (npairs) *npairs = p->npairs;
    if (depth_D) *depth_D = p->depth_D;
    if (levels_lower) *levels_lower = p->levels[0];
    if (levels_upper) *levels_upper = p->levels[1];
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
