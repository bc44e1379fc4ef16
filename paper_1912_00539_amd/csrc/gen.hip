// Seeded synthetic 4x4-block Jacobians generated on the device (the serving benchmark's input
// source). Structure and random keys follow the host generator; no preconditioner arithmetic.
#include "setup_kernels.h"

using namespace abilu;
using namespace abilu_dev;

namespace {

using namespace abilu_setup;

template <int KIND>
__global__ void k_gen_rowlen(int nx, int ny, uint64_t seed, int n, int64_t *len) {
    gen_rowlen_body<KIND>(blockIdx.x, nx, ny, seed, n, len);
}

template <int KIND>
__global__ __launch_bounds__(WG) void k_gen_fill(int nx, int ny, double cfl, uint64_t seed, int n,
                                                 const int32_t *__restrict__ rowptr, int32_t *__restrict__ colidx,
                                                 double *__restrict__ A, double *__restrict__ b) {
    gen_fill_body<KIND>(blockIdx.x, nx, ny, cfl, seed, n, rowptr, colidx, A, b);
}

bool sizes_of(const abilu_gen_spec *s, int64_t *n, int64_t *z) {
    if (!s || s->nx < 1 || s->ny < 1 || !(s->cfl > 0.0)) return false;
    const int64_t nx = s->nx, ny = s->ny;
    if (s->kind == ABILU_GEN_TRI) {
        const int64_t nq = nx * ny, F = nq + ny * (nx - 1) + (ny - 1) * nx;
        *n = 2 * nq;
        *z = *n + 2 * F;
    } else if (s->kind == ABILU_GEN_ANISO) {
        const int64_t F = ny * (nx - 1) + (ny - 1) * nx;
        *n = nx * ny;
        *z = *n + 2 * F;
    } else {
        return false;
    }
    return *n < (int64_t)1 << 30 && *z < (int64_t)1 << 31;
}

}  // namespace

extern "C" abilu_status abilu_gen_sizes(const abilu_gen_spec *spec, int32_t *n, int64_t *nnzb) {
    int64_t nn, zz;
    if (!sizes_of(spec, &nn, &zz)) return ABILU_EINVAL;
    if (n) *n = (int32_t)nn;
    if (nnzb) *nnzb = zz;
    return ABILU_OK;
}

extern "C" size_t abilu_gen_scratch_bytes(const abilu_gen_spec *spec) {
    int64_t nn, zz;
    if (!sizes_of(spec, &nn, &zz)) return 0;
    return sizeof(int64_t) * (size_t)((nn + 1) + scan_tiles(nn) + 1);
}

extern "C" abilu_status abilu_gen_build(const abilu_gen_spec *spec, int32_t *d_rowptr, int32_t *d_colidx,
                                        double *d_A, double *d_b, void *d_scratch, void *stream) {
    int64_t nn, zz;
    if (!sizes_of(spec, &nn, &zz)) return ABILU_EINVAL;
    if (!d_rowptr || !d_colidx || !d_A || !d_b || !d_scratch) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)nn;
    int64_t *len = (int64_t *)d_scratch;
    int64_t *tot = len + (nn + 1);
    {
        ProfScope ps("gen_rowlen", s, 8.0 * nn);
        if (spec->kind == ABILU_GEN_TRI)
            k_gen_rowlen<ABILU_GEN_TRI><<<div_up(n, 256), 256, 0, s>>>(spec->nx, spec->ny, spec->seed, n, len);
        else
            k_gen_rowlen<ABILU_GEN_ANISO><<<div_up(n, 256), 256, 0, s>>>(spec->nx, spec->ny, spec->seed, n, len);
    }
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    if (!hip_ok(scan_exclusive(nn, len, tot, nullptr, d_rowptr, s), "gen rowptr scan")) return ABILU_EDEVICE;
    {
        ProfScope ps("gen_fill", s, 4.0 * (nn + 1) + 132.0 * zz + 32.0 * nn);
        if (spec->kind == ABILU_GEN_TRI)
            k_gen_fill<ABILU_GEN_TRI><<<div_up(n, ROWS_PER_WG), WG, 0, s>>>(spec->nx, spec->ny, spec->cfl, spec->seed, n,
                                                                           d_rowptr, d_colidx, d_A, d_b);
        else
            k_gen_fill<ABILU_GEN_ANISO><<<div_up(n, ROWS_PER_WG), WG, 0, s>>>(spec->nx, spec->ny, spec->cfl, spec->seed,
                                                                             n, d_rowptr, d_colidx, d_A, d_b);
    }
    return launch_status();
}
