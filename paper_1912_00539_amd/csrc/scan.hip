// Exclusive prefix sums of int64 counts on the device (3 phases: per-tile scan, scan of the
// tile totals in one workgroup, add of each tile's offset), used by the pattern analysis, the
// chunk schedules and the request generator.
#include "setup_kernels.h"

namespace {

using namespace abilu_setup;

__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(int64_t len, const int64_t *__restrict__ in,
                                                       int64_t *__restrict__ out, int64_t *__restrict__ tot) {
    scan_tiles_body(blockIdx.x, len, in, out, tot);
}

__global__ __launch_bounds__(SCAN_T) void k_scan_totals(int ntiles, int64_t *__restrict__ tot,
                                                        int64_t *__restrict__ grand) {
    scan_totals_body(ntiles, tot, grand);
}

__global__ __launch_bounds__(SCAN_T) void k_scan_finish(int64_t len, const int64_t *__restrict__ scan, const int64_t *__restrict__ tot,
                              const int64_t *__restrict__ grand, int64_t *__restrict__ ptr64,
                              int32_t *__restrict__ ptr32) {
    scan_finish_body(blockIdx.x, len, scan, tot, grand, ptr64, ptr32);
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
    k_scan_finish<<<div_up(len + 1, SCAN_TILE), SCAN_T, 0, s>>>(len, tmp, tot, tot + nt, out64, out32);
    return hipGetLastError();
}

}  // namespace abilu
