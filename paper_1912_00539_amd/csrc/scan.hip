// Exclusive prefix sums of int64 counts on the device (3 phases: per-tile sums, scan of the
// tile sums in one workgroup, each tile scanned from its offset), used by the pattern analysis,
// the chunk schedules and the request generator.
#include "setup_kernels.h"

namespace {

using namespace abilu_setup;

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(int64_t len, const int64_t *__restrict__ in,
                                                        int64_t *__restrict__ tot) {
    scan_reduce_body(blockIdx.x, len, in, tot);
}

__global__ __launch_bounds__(SCAN_T) void k_scan_totals(int ntiles, int64_t *__restrict__ tot,
                                                        int64_t *__restrict__ grand) {
    scan_totals_body(ntiles, tot, grand);
}

__global__ __launch_bounds__(SCAN_T) void k_scan_finish(int64_t len, const int64_t *__restrict__ in,
                                                        const int64_t *__restrict__ tot,
                                                        const int64_t *__restrict__ grand,
                                                        int64_t *__restrict__ ptr64, int32_t *__restrict__ ptr32) {
    scan_finish_body(blockIdx.x, len, in, tot, grand, ptr64, ptr32);
}

}  // namespace

namespace abilu {

int scan_tiles(int64_t len) { return div_up(len > 0 ? len : 1, SCAN_TILE); }

hipError_t scan_exclusive(int64_t len, const int64_t *in, int64_t *tot, int64_t *out64, int32_t *out32,
                          hipStream_t s) {
    const int nt = scan_tiles(len);
    k_scan_reduce<<<nt, SCAN_T, 0, s>>>(len, in, tot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_scan_totals<<<1, SCAN_T, 0, s>>>(nt, tot, tot + nt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_finish<<<div_up(len + 1, SCAN_TILE), SCAN_T, 0, s>>>(len, in, tot, tot + nt, out64, out32);
    return hipGetLastError();
}

}  // namespace abilu
