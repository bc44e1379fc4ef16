// Dependency depth of the block ILU fixed-point problem (Lemma 2 and Theorem 8, Section 4.2) and
// the levels of the two block triangular solves (Theorem 3, Section 4.1), on the device.
//
// Both are longest-path lengths over an acyclic dependence graph whose topological order is the
// row order (the Gaussian-elimination ordering of the blocks for the depth, ascending rows for the
// lower levels, descending rows for the upper levels). They are computed by monotone relaxation:
// every value starts at 0, below its fixed point, and a pass sets each value to 1 + the largest of
// the values it depends on as they are in memory at the time, never lowering it. By induction over
// the topological order, no value ever exceeds its fixed point, and a pass that changes nothing
// leaves every value equal to 1 + the largest of its dependencies, i.e. at the fixed point. Passes
// update in place, so a read may see a value of the same pass or an older one; either is below or
// at the fixed point, and only the number of passes depends on which.
//
// One thread per row: row t's blocks in ascending column order (a block reads the X_ik of its own
// row, computed earlier in the same pass) and its lower level, and the upper level of row n-1-t,
// so that both chains run with the ascending dispatch order of the workgroups. After the first
// pass a row is recomputed only when it or a row it reads changed in the pass before: at the fixed
// point every row was recomputed after the last change of everything it reads, and most passes
// touch only the rows near the advancing front of the longest chains.
#include "abilu_internal.h"

using namespace abilu;

namespace {

constexpr int DWG = 256;
constexpr int BATCH = 32;   // passes launched between two host checks

// One relaxation pass. A row is recomputed only if it, or a row it reads, changed in the previous
// pass (chg_prev): the lower rows for its blocks' depths and its lower level, the upper rows for
// its upper level. Rows that change raise chg_cur; chg_clear (the flags two passes on) is zeroed
// here, so that three flag arrays rotate without a separate clearing launch.
__global__ __launch_bounds__(DWG) void k_depth_pass(int n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ colidx,
                                                    const int32_t *__restrict__ diag_pos,
                                                    const int32_t *__restrict__ pair_ptr,
                                                    const int32_t *__restrict__ pik, const int32_t *__restrict__ pkj,
                                                    int32_t *depth, int32_t *lev_l, int32_t *lev_u,
                                                    const uint8_t *__restrict__ chg_prev, uint8_t *chg_cur,
                                                    uint8_t *__restrict__ chg_clear, int all, int *changed) {
    const int t = blockIdx.x * DWG + threadIdx.x;
    bool ch = false;
    if (t < n) {
        chg_clear[t] = 0;
        const int i = t;
        const int b0 = rowptr[i], d = diag_pos[i];
        bool go = all || chg_prev[i];
        for (int e = b0; e < d && !go; ++e) go = chg_prev[colidx[e]] != 0;
        if (go) {
            bool mine = false;
            int ml = 0;
            for (int e = b0; e < rowptr[i + 1]; ++e) {
                const int j = colidx[e];
                int dd = 0;
                for (int q = pair_ptr[e]; q < pair_ptr[e + 1]; ++q) dd = max(dd, max(depth[pik[q]], depth[pkj[q]]));
                if (i > j) {
                    dd = max(dd, depth[diag_pos[j]]);
                    ml = max(ml, lev_l[j]);
                }
                if (dd + 1 > depth[e]) {
                    depth[e] = dd + 1;
                    mine = true;
                }
            }
            if (ml + 1 > lev_l[i]) {
                lev_l[i] = ml + 1;
                mine = true;
            }
            if (mine) {
                chg_cur[i] = 1;
                ch = true;
            }
        }
        const int iu = n - 1 - t;
        const int du = diag_pos[iu], e1 = rowptr[iu + 1];
        bool gu = all || chg_prev[iu];
        for (int e = du + 1; e < e1 && !gu; ++e) gu = chg_prev[colidx[e]] != 0;
        if (gu) {
            int mu = 0;
            for (int e = du + 1; e < e1; ++e) mu = max(mu, lev_u[colidx[e]]);
            if (mu + 1 > lev_u[iu]) {
                lev_u[iu] = mu + 1;
                chg_cur[iu] = 1;
                ch = true;
            }
        }
    }
    // one flag write per wavefront that changed something
    if (__any(ch) && (threadIdx.x & 63) == 0) atomicOr(changed, 1);
}

__global__ __launch_bounds__(DWG) void k_fill_i32(int64_t len, int32_t *v, int32_t val) {
    const int64_t t = (int64_t)blockIdx.x * DWG + threadIdx.x;
    if (t < len) v[t] = val;
}

// out[0] = max depth, out[1] = max lower level, out[2] = max upper level (out zeroed before)
__global__ __launch_bounds__(DWG) void k_depth_max(int64_t Z, int n, const int32_t *__restrict__ depth,
                                                   const int32_t *__restrict__ lev_l,
                                                   const int32_t *__restrict__ lev_u, int *out) {
    int md = 0, ml = 0, mu = 0;
    const int64_t stride = (int64_t)gridDim.x * DWG;
    for (int64_t t = (int64_t)blockIdx.x * DWG + threadIdx.x; t < Z; t += stride) md = max(md, depth[t]);
    for (int64_t t = (int64_t)blockIdx.x * DWG + threadIdx.x; t < n; t += stride) {
        ml = max(ml, lev_l[t]);
        mu = max(mu, lev_u[t]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        md = max(md, __shfl_xor(md, o, 64));
        ml = max(ml, __shfl_xor(ml, o, 64));
        mu = max(mu, __shfl_xor(mu, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(out, md);
        atomicMax(out + 1, ml);
        atomicMax(out + 2, mu);
    }
}

}  // namespace

extern "C" abilu_status abilu_pattern_depth(abilu_pattern *p, int32_t *d_depth, int32_t *d_level_lower,
                                            int32_t *d_level_upper, int32_t *depth_D, int32_t *levels_lower,
                                            int32_t *levels_upper, void *stream) {
    if (!p) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = p->n;
    const int64_t Z = p->nnzb;
    if (n == 0) {
        p->depth_D = 0;
        p->levels[0] = p->levels[1] = 0;
    } else {
        // scratch: depth[Z], lev_l[N], lev_u[N], BATCH pass flags, 3 maxima, then 3 x N row flags
        int32_t *buf = nullptr;
        const size_t words = (size_t)Z + 2 * (size_t)n + BATCH + 3;
        const size_t rowflags = ((size_t)3 * n + 3) / 4;     // in int32 words
        if (!hip_ok(hipMalloc(&buf, sizeof(int32_t) * (words + rowflags)), "depth scratch")) return ABILU_ENOMEM;
        int32_t *depth = buf, *lev_l = buf + Z, *lev_u = lev_l + n, *flags = lev_u + n, *mx = flags + BATCH;
        uint8_t *chg = (uint8_t *)(buf + words);
        abilu_status st = ABILU_OK;
        const int grid = div_up(n, DWG);
        // each pass reads at least the values the pass before it left, so after pass p every value
        // whose longest dependence chain has at most p links is final: the relaxation settles
        // within max(D, levels) + 1 <= Z + 1 passes. The cap only guards against a fault.
        const int64_t cap = Z + (int64_t)n + 2 * BATCH;
        int64_t passes = 0;
        bool done = false;
        k_fill_i32<<<div_up((int64_t)(words + rowflags), DWG), DWG, 0, s>>>((int64_t)(words + rowflags), buf, 0);
        if (launch_status() != ABILU_OK) st = ABILU_EDEVICE;
        while (st == ABILU_OK && !done) {
            k_fill_i32<<<1, DWG, 0, s>>>(BATCH, flags, 0);
            for (int q = 0; q < BATCH; ++q) {
                const int64_t pass = passes + q;
                k_depth_pass<<<grid, DWG, 0, s>>>(n, p->rowptr, p->colidx, p->diag_pos, p->pair_ptr, p->pik, p->pkj,
                                                   depth, lev_l, lev_u, chg + (size_t)n * ((pass + 2) % 3),
                                                   chg + (size_t)n * (pass % 3), chg + (size_t)n * ((pass + 1) % 3),
                                                   pass == 0 ? 1 : 0, flags + q);
            }
            if (launch_status() != ABILU_OK) { st = ABILU_EDEVICE; break; }
            int32_t h[BATCH];
            if (!hip_ok(hipMemcpyAsync(h, flags, sizeof h, hipMemcpyDeviceToHost, s), "depth flags") ||
                !hip_ok(hipStreamSynchronize(s), "depth flags sync")) {
                st = ABILU_EDEVICE;
                break;
            }
            for (int q = 0; q < BATCH; ++q) done = done || h[q] == 0;
            passes += BATCH;
            if (!done && passes > cap) {
                note_error("depth relaxation did not settle within the bound on its passes");
                st = ABILU_EDEVICE;
            }
        }
        if (st == ABILU_OK) {
            k_depth_max<<<div_up(Z > n ? Z : n, DWG * 8), DWG, 0, s>>>(Z, n, depth, lev_l, lev_u, mx);
            int32_t h[3] = {0, 0, 0};
            hipError_t e = hipGetLastError();
            if (e == hipSuccess && d_depth) e = hipMemcpyAsync(d_depth, depth, sizeof(int32_t) * Z, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && d_level_lower)
                e = hipMemcpyAsync(d_level_lower, lev_l, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && d_level_upper)
                e = hipMemcpyAsync(d_level_upper, lev_u, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(h, mx, sizeof h, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (!hip_ok(e, "depth results")) {
                st = ABILU_EDEVICE;
            } else {
                p->depth_D = h[0];
                p->levels[0] = h[1];
                p->levels[1] = h[2];
            }
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        if (st != ABILU_OK) return st;
    }
    if (depth_D) *depth_D = p->depth_D;
    if (levels_lower) *levels_lower = p->levels[0];
    if (levels_upper) *levels_upper = p->levels[1];
    return ABILU_OK;
}
