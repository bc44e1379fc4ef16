// Chunk schedules for the chunked sweeps. The paper's implementation hands each worker a chunk of
// consecutive rows, which it runs in row-major order (Section 3.3), so that within a chunk the
// blocks are computed in a Gaussian-elimination ordering. Here one workgroup runs one chunk: row i
// of the chunk only reads values of the chunk's rows k < i that are its strictly lower neighbours
// (the L_ik of its own row, and U_kj, U_kk^{-1} of rows k with (i,k) in S_B), so the rows can be
// taken level by level, where the level of a row is one more than the largest level among its
// lower neighbours in the chunk, with a workgroup barrier between levels; this gives exactly the
// values of the sequential row-major order. The backward apply sweep runs a chunk's rows in
// descending order and uses the same construction on the upper neighbours.
#include "abilu_internal.h"

namespace {

using namespace abilu;

// One thread per chunk: levels of the chunk's rows in the lower graph (rows ascending) and the
// upper graph (rows descending), the number of entries each chunk needs in lvstart (levels + 1)
// and the largest level counts.
__global__ void k_chunk_levels(int n, int R, int nch, const int32_t *__restrict__ rowptr,
                               const int32_t *__restrict__ colidx, const int32_t *__restrict__ diag_pos,
                               int32_t *lev_lo, int32_t *lev_up, int64_t *__restrict__ cnt_lo,
                               int64_t *__restrict__ cnt_up, int *__restrict__ maxlev) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch) return;
    const int c0 = c * R, c1 = min(n, c0 + R);
    int ml = 0;
    for (int i = c0; i < c1; ++i) {
        int l = 0;
        for (int e = rowptr[i]; e < diag_pos[i]; ++e) {
            const int k = colidx[e];
            if (k >= c0) l = max(l, lev_lo[k]);
        }
        lev_lo[i] = l + 1;
        ml = max(ml, l + 1);
    }
    int mu = 0;
    for (int i = c1 - 1; i >= c0; --i) {
        int l = 0;
        for (int e = diag_pos[i] + 1; e < rowptr[i + 1]; ++e) {
            const int j = colidx[e];
            if (j < c1) l = max(l, lev_up[j]);
        }
        lev_up[i] = l + 1;
        mu = max(mu, l + 1);
    }
    cnt_lo[c] = ml + 1;
    cnt_up[c] = mu + 1;
    atomicMax(&maxlev[0], ml);
    atomicMax(&maxlev[1], mu);
}

// One workgroup per chunk: the chunk's rows sorted by level (ascending rows within a level), and
// the start of every level followed by the chunk's end. Levels run 1..L without gaps (a row of
// level l > 1 has a lower neighbour of level l - 1), so each level's first row records its start.
__global__ __launch_bounds__(256) void k_chunk_order(int n, int R, const int32_t *__restrict__ lev,
                                                     const int32_t *__restrict__ lvptr,
                                                     int32_t *__restrict__ order, int32_t *__restrict__ lvstart) {
    __shared__ int sl[MAX_CHUNK_ROWS];
    const int c = blockIdx.x, c0 = c * R, c1 = min(n, c0 + R), m = c1 - c0;
    for (int t = threadIdx.x; t < m; t += blockDim.x) sl[t] = lev[c0 + t];
    __syncthreads();
    const int b = lvptr[c];
    const int nl = lvptr[c + 1] - b - 1;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int lt = sl[t];
        int before = 0, rank = 0;
        for (int q = 0; q < m; ++q) {
            const int lq = sl[q];
            before += (lq < lt) ? 1 : 0;
            rank += (lq == lt && q < t) ? 1 : 0;
        }
        order[c0 + before + rank] = c0 + t;
        if (rank == 0) lvstart[b + lt - 1] = c0 + before;
    }
    if (threadIdx.x == 0) lvstart[b + nl] = c1;
}

// The record of row i (layout beside REC_INTS), written to `out`; returns the row's counts of
// strictly lower and upper blocks and update pairs.
__device__ void chunk_record(int i, int n, int R, int ZL, const int32_t *__restrict__ rowptr,
                             const int32_t *__restrict__ colidx, const int32_t *__restrict__ diag_pos,
                             const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
                             const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ sik,
                             const int32_t *__restrict__ skj, const int32_t *__restrict__ pkj,
                             int32_t *__restrict__ rec, int64_t idx, int64_t nr, int (&counts)[3]) {
    // field k of this record: component k % 4 of entry idx of plane k / 4
    auto put = [&](int k, int v) { rec[((int64_t)(k >> 2) * nr + idx) * 4 + (k & 3)] = v; };
    const int c0 = (i / R) * R, c1 = min(n, c0 + R);
    const int b0 = rowptr[i], b1 = rowptr[i + 1], d = diag_pos[i];
    const int nl = d - b0, nu = b1 - d - 1;
    const int p0 = pair_ptr[b0], np = pair_ptr[b1] - p0;
    for (int k = 0; k < REC_INTS; ++k) put(k, 0);
    put(0, b0);
    put(1, lrow[i]);
    put(2, urow[i]);
    int meta = min(nl, 15) | (min(nu, 15) << 4) | (min(np, 15) << 8);
    for (int u = 0; u < min(nl, REC_CAP); ++u) {
        const int j = colidx[b0 + u];
        const int src = j < c0 ? REC_OUT : (j == i - 1 ? REC_PREV : REC_CHUNK);
        meta |= src << (12 + 2 * u);
        put(4 + u, j);
    }
    for (int w = 0; w < min(nu, REC_CAP); ++w) {
        const int j = colidx[d + 1 + w];
        const int src = j >= c1 ? REC_OUT : (j == i + 1 ? REC_PREV : REC_CHUNK);
        meta |= src << (20 + 2 * w);
        put(20 + w, j);
    }
    put(3, meta);
    // U_kj at factor-layout position s belongs to a row of the chunk when s >= ubound, to row i - 1
    // when s lies in that row's upper part
    const int ubase = ZL + n;
    const int ubound = ubase + urow[c0];
    const int prev0 = i > c0 ? ubase + urow[i - 1] : -1, prev1 = ubase + urow[i];
    int e = b0;
    for (int q = 0; q < min(np, REC_CAP); ++q) {
        const int pq = p0 + q;
        while (pair_ptr[e + 1] <= pq) ++e;   // the block the pair updates
        const int tgt = e < d ? e - b0 : (e == d ? 4 : 5 + (e - d - 1));
        const int lord = sik[pq] - lrow[i];
        const int sp = skj[pq];
        int src = REC_OUT, o = 0;
        if (sp >= ubound) {
            src = REC_CHUNK;
            if (prev0 >= 0 && sp >= prev0 && sp < prev1) {
                // row i - 1: its blocks are in registers when it had at most REC_CAP upper blocks
                src = REC_PREV;
                o = (sp - prev0) & 3;
            }
        }
        put(8 + q, (tgt & 15) | ((lord & 3) << 4) | (src << 6) | (o << 8));
        put(12 + q, sp);
        put(16 + q, pkj[pq]);
    }
    counts[0] = nl;
    counts[1] = nu;
    counts[2] = np;
}

// One thread per row: the records (planes of int4, each step-major: row c * R + t at index
// t * nch + c), and the largest counts of a row (one atomic per wavefront).
__global__ void k_chunk_records(int n, int R, int nch, int ZL, const int32_t *__restrict__ rowptr,
                                const int32_t *__restrict__ colidx, const int32_t *__restrict__ diag_pos,
                                const int32_t *__restrict__ lrow, const int32_t *__restrict__ urow,
                                const int32_t *__restrict__ pair_ptr, const int32_t *__restrict__ sik,
                                const int32_t *__restrict__ skj, const int32_t *__restrict__ pkj,
                                int32_t *__restrict__ rec, int *__restrict__ maxima) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int mx[3] = {0, 0, 0};
    if (i < n) {
        const int c = i / R, t = i - c * R;
        chunk_record(i, n, R, ZL, rowptr, colidx, diag_pos, lrow, urow, pair_ptr, sik, skj, pkj, rec,
                     (int64_t)t * nch + c, (int64_t)R * nch, mx);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx[q] = max(mx[q], __shfl_xor(mx[q], o, 64));
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 3; ++q) atomicMax(&maxima[q], mx[q]);
}

}  // namespace

namespace abilu {

// AUTO: a quad per chunk when the chunks are close to chains (few rows per dependence level: a
// workgroup per chunk would keep most of its quads idle at every level), otherwise a workgroup per
// chunk taking each level's rows in parallel.
int32_t chunk_runner_auto(int n, int nch, const int64_t *total_levels) {
    const int64_t lv = total_levels[0] > total_levels[1] ? total_levels[0] : total_levels[1];
    return (double)n / (double)(lv > 0 ? lv : 1) < 4.0 ? ABILU_CHUNK_BY_ROWS : ABILU_CHUNK_BY_LEVELS;
}

void free_chunks(abilu_pattern *p) {
    for (int s = 0; s < 2; ++s) {
        (void)hipFree(p->order[s]);
        (void)hipFree(p->lvptr[s]);
        (void)hipFree(p->lvstart[s]);
        p->order[s] = p->lvptr[s] = p->lvstart[s] = nullptr;
        p->max_levels[s] = 0;
        p->total_levels[s] = 0;
    }
    (void)hipFree(p->rec);
    p->rec = nullptr;
    p->rec_max[0] = p->rec_max[1] = p->rec_max[2] = 0;
    p->chunk_rows = 0;
    p->nchunks = 0;
    p->chunk_runner = 0;
}

}  // namespace abilu

extern "C" abilu_status abilu_pattern_set_chunks(abilu_pattern *p, int32_t rows_per_chunk, int32_t runner,
                                                 void *stream) {
    using namespace abilu;
    if (!p || rows_per_chunk < 1 || rows_per_chunk > MAX_CHUNK_ROWS) return ABILU_EINVAL;
    if (runner != ABILU_CHUNK_AUTO && runner != ABILU_CHUNK_BY_LEVELS && runner != ABILU_CHUNK_BY_ROWS)
        return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    free_chunks(p);
    const int n = p->n, R = rows_per_chunk;
    if (n == 0) {
        p->chunk_rows = R;
        p->chunk_runner = runner == ABILU_CHUNK_AUTO ? ABILU_CHUNK_BY_LEVELS : runner;
        return ABILU_OK;
    }
    const int nch = div_up(n, R);
    abilu_status st = ABILU_OK;
    char *scratch = nullptr;
    // scratch: lev[2][n], cnt[2][nch + 1], scan tiles, maxlev[2]
    const size_t o_lev = 0;
    const size_t o_cnt = o_lev + 256 * (size_t)div_up(2 * sizeof(int32_t) * (size_t)n, 256);
    const size_t o_tot = o_cnt + 2 * sizeof(int64_t) * (size_t)(nch + 1);
    const size_t o_max = o_tot + sizeof(int64_t) * (size_t)(scan_tiles(nch) + 1);
    const size_t sbytes = o_max + 64;
    int32_t *lev = nullptr;
    int64_t *cnt = nullptr, *tot = nullptr;
    int *maxlev = nullptr;
    int32_t *h = (int32_t *)p->pinned;
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
    CKA(hipMalloc(&scratch, sbytes));
    lev = (int32_t *)(scratch + o_lev);
    cnt = (int64_t *)(scratch + o_cnt);
    tot = (int64_t *)(scratch + o_tot);
    maxlev = (int *)(scratch + o_max);
    for (int q = 0; q < 2; ++q) {
        CKA(hipMalloc(&p->order[q], sizeof(int32_t) * (size_t)n));
        CKA(hipMalloc(&p->lvptr[q], sizeof(int32_t) * (size_t)(nch + 1)));
    }
    CK(hipMemsetAsync(maxlev, 0, 2 * sizeof(int), s));
    k_chunk_levels<<<div_up(nch, 256), 256, 0, s>>>(n, R, nch, p->rowptr, p->colidx, p->diag_pos, lev, lev + n,
                                                   cnt, cnt + (nch + 1), maxlev);
    CK(hipGetLastError());
    for (int q = 0; q < 2; ++q) {
        CK(scan_exclusive(nch, cnt + q * (nch + 1), tot, nullptr, p->lvptr[q], s));
        CK(hipMemcpyAsync(h + q, p->lvptr[q] + nch, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    CK(hipMemcpyAsync(h + 2, maxlev, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    for (int q = 0; q < 2; ++q) {
        p->total_levels[q] = (int64_t)h[q] - nch;
        p->max_levels[q] = h[2 + q];
        CKA(hipMalloc(&p->lvstart[q], sizeof(int32_t) * (size_t)h[q]));
    }
    for (int q = 0; q < 2; ++q) {
        k_chunk_order<<<nch, 256, 0, s>>>(n, R, lev + (size_t)q * n, p->lvptr[q], p->order[q], p->lvstart[q]);
        CK(hipGetLastError());
    }
    CK(hipStreamSynchronize(s));
    (void)hipFree(scratch);
    scratch = nullptr;
    p->chunk_runner = runner != ABILU_CHUNK_AUTO ? runner : chunk_runner_auto(n, nch, p->total_levels);
    if (p->chunk_runner == ABILU_CHUNK_BY_ROWS) {
        // the records, then the largest lower, upper and pair counts of a row
        const size_t rbytes = sizeof(int32_t) * REC_INTS * (size_t)nch * (size_t)R;
        CKA(hipMalloc(&p->rec, rbytes + 4 * sizeof(int)));
        int *maxima = (int *)((char *)p->rec + rbytes);
        CK(hipMemsetAsync(maxima, 0, 4 * sizeof(int), s));
        k_chunk_records<<<div_up(n, 256), 256, 0, s>>>(n, R, nch, (int)p->nnzb_lower, p->rowptr, p->colidx,
                                                       p->diag_pos, p->lrow, p->urow, p->pair_ptr, p->sik, p->skj,
                                                       p->pkj, p->rec, maxima);
        CK(hipGetLastError());
        CK(hipMemcpyAsync(h, maxima, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        for (int q = 0; q < 3; ++q) p->rec_max[q] = h[q];
    }
    p->chunk_rows = R;
    p->nchunks = nch;
    return ABILU_OK;
fail:
    (void)hipStreamSynchronize(s);
    (void)hipFree(scratch);
    free_chunks(p);
    return st;
#undef CK
#undef CKA
}

extern "C" abilu_status abilu_pattern_chunk_info(const abilu_pattern *p, int32_t *rows_per_chunk, int32_t *nchunks,
                                                 int32_t *runner, int32_t *max_levels_lower,
                                                 int32_t *max_levels_upper, int64_t *levels_lower,
                                                 int64_t *levels_upper) {
    if (!p) return ABILU_EINVAL;
    if (runner) *runner = p->chunk_rows ? p->chunk_runner : 0;
    if (rows_per_chunk) *rows_per_chunk = p->chunk_rows;
    if (nchunks) *nchunks = p->nchunks;
    if (max_levels_lower) *max_levels_lower = p->max_levels[0];
    if (max_levels_upper) *max_levels_upper = p->max_levels[1];
    if (levels_lower) *levels_lower = p->total_levels[0];
    if (levels_upper) *levels_upper = p->total_levels[1];
    return ABILU_OK;
}

extern "C" abilu_status abilu_pattern_chunk_export(const abilu_pattern *p, int32_t upper, int32_t *d_order,
                                                   int32_t *d_lvptr, int32_t *d_lvstart, void *stream) {
    if (!p || (upper != 0 && upper != 1)) return ABILU_EINVAL;
    if (p->chunk_rows == 0) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int q = upper;
    hipError_t e = hipSuccess;
    if (d_order && p->n > 0)
        e = hipMemcpyAsync(d_order, p->order[q], sizeof(int32_t) * (size_t)p->n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_lvptr && p->nchunks > 0)
        e = hipMemcpyAsync(d_lvptr, p->lvptr[q], sizeof(int32_t) * (size_t)(p->nchunks + 1), hipMemcpyDeviceToDevice,
                           s);
    if (e == hipSuccess && d_lvstart && p->nchunks > 0)
        e = hipMemcpyAsync(d_lvstart, p->lvstart[q], sizeof(int32_t) * (size_t)(p->total_levels[q] + p->nchunks),
                           hipMemcpyDeviceToDevice, s);
    return abilu::hip_ok(e, "chunk schedule export copy") ? ABILU_OK : ABILU_EDEVICE;
}
