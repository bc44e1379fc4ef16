// Exclusive prefix sums of int64 counts on the device (3 phases: per-tile scan, scan of the
// tile totals in one workgroup, add), used by the pattern analysis and the request generator.
#include "abilu_internal.h"

namespace {

constexpr int SCAN_T = 256, SCAN_E = 8, SCAN_TILE = SCAN_T * SCAN_E;

__device__ long long block_exclusive(long long v, long long *sh, long long *total) {
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

__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(int64_t len, const int64_t *__restrict__ in,
                                                       int64_t *__restrict__ out, int64_t *__restrict__ tot) {
    __shared__ long long sh[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_E;
    long long v[SCAN_E], s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_E; ++q) {
        v[q] = (base + q < len) ? in[base + q] : 0;
        s += v[q];
    }
    long long total;
    long long pre = block_exclusive(s, sh, &total);
#pragma unroll
    for (int q = 0; q < SCAN_E; ++q) {
        if (base + q < len) out[base + q] = pre;
        pre += v[q];
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_totals(int ntiles, int64_t *__restrict__ tot,
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

__global__ void k_scan_finish(int64_t len, const int64_t *__restrict__ scan, const int64_t *__restrict__ tot,
                              const int64_t *__restrict__ grand, int64_t *__restrict__ ptr64,
                              int32_t *__restrict__ ptr32) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) {
        int64_t v = scan[e] + tot[e / SCAN_TILE];
        if (ptr64) ptr64[e] = v;
        ptr32[e] = (int32_t)v;
    } else if (e == len) {
        if (ptr64) ptr64[len] = *grand;
        ptr32[len] = (int32_t)*grand;
    }
}

}  // namespace

namespace abilu {

int scan_tiles(int64_t len) { return div_up(len > 0 ? len : 1, SCAN_TILE); }

hipError_t scan_exclusive(int64_t len, const int64_t *in, int64_t *tmp, int64_t *tot, int64_t *out64,
                          int32_t *out32, hipStream_t s) {
    const int nt = scan_tiles(len);
    k_scan_tiles<<<nt, SCAN_T, 0, s>>>(len, in, tmp, tot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_scan_totals<<<1, SCAN_T, 0, s>>>(nt, tot, tot + nt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_finish<<<div_up(len + 1, 256), 256, 0, s>>>(len, tmp, tot, tot + nt, out64, out32);
    return hipGetLastError();
}

}  // namespace abilu
