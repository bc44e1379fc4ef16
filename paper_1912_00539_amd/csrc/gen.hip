// Seeded synthetic 4x4-block Jacobians generated on the device (the serving benchmark's input
// source). Structure and random keys follow the host generator; no preconditioner arithmetic.
#include <climits>
#include <cmath>

#include "abilu_gen.h"
#include "abilu_internal.h"

using namespace abilu;
using namespace abilu_dev;

namespace {

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr uint64_t STREAM_MUL = 0xD1B54A32D192ED03ull;
enum { S_FACE_W = 1, S_OFFDIAG = 2, S_DIAGPERT = 3, S_RHS = 4, S_SPLIT = 5 };

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}
__device__ inline uint64_t key(uint64_t seed, uint64_t stream) { return mix64(seed * GOLDEN + stream * STREAM_MUL); }
__device__ inline double u01(uint64_t k, uint64_t idx) {
    return (double)(mix64(k + idx * GOLDEN) >> 11) * (1.0 / 9007199254740992.0);
}
// lo + (hi - lo) u without a fused multiply-add, like the host generator
__device__ inline double uab(uint64_t k, uint64_t idx, double lo, double hi) {
    return __dadd_rn(lo, __dmul_rn(hi - lo, u01(k, idx)));
}

// Neighbours of a cell in four fixed slots (absent ones have col = -1), as separate scalar
// arrays indexed by compile-time constants so that they stay in registers.
struct Nbs {
    int col[4];       // neighbour cell (output numbering), -1: none
    int64_t face[4];  // natural face index
    int dir[4];       // 0: this cell is the face's first cell (counter 2f), 1: second (2f + 1)
    double scale[4];  // face weight factor (anisotropy)
};

__device__ __forceinline__ void set_nb(Nbs &b, int q, int col, int64_t face, int dir, double scale) {
    b.col[q] = col;
    b.face[q] = face;
    b.dir[q] = dir;
    b.scale[q] = scale;
}

__device__ __forceinline__ bool tri_diag(uint64_t ksplit, int q) { return u01(ksplit, (uint64_t)q) < 0.5; }  // '\'

template <int KIND>
__device__ __forceinline__ void neighbours(int nx, int ny, uint64_t ksplit, int c, int *nat, Nbs &b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) set_nb(b, q, -1, 0, 0, 1.0);
    if constexpr (KIND == ABILU_GEN_TRI) {
        // natural order: cell 2q + t, quad q = iy*nx + ix
        const int q = c >> 1, t = c & 1, ix = q % nx, iy = q / nx;
        const int64_t nq = (int64_t)nx * ny;
        const bool dq = tri_diag(ksplit, q);
        *nat = c;
        // diagonal face q: first cell 2q, second 2q+1
        set_nb(b, 0, t == 0 ? 2 * q + 1 : 2 * q, (int64_t)q, t, 1.0);
        const int64_t hface_l = nq + (int64_t)iy * (nx - 1) + (ix - 1);   // left edge of the quad
        const int64_t hface_r = nq + (int64_t)iy * (nx - 1) + ix;         // right edge
        // the triangle on the left edge of quad q (second cell of that face) or on its right edge
        // (first cell); the neighbour across is the right / left owner of the adjacent quad.
        // Each slot is written once, from selected values.
        const bool on_left = (t == 0) == dq;
        if (on_left ? ix > 0 : ix < nx - 1) {
            const int qq = on_left ? q - 1 : q + 1;
            const bool dd = tri_diag(ksplit, qq);
            const int col = (on_left == dd) ? 2 * qq + 1 : 2 * qq;
            set_nb(b, 2, col, on_left ? hface_l : hface_r, on_left ? 1 : 0, 1.0);
        }
        // bottom edge (t = 0, second cell of the face below) or top edge (t = 1, first cell)
        if (t == 0 ? iy > 0 : iy < ny - 1) {
            const int row = t == 0 ? iy - 1 : iy;
            set_nb(b, 1, t == 0 ? 2 * (q - nx) + 1 : 2 * (q + nx), nq + (int64_t)ny * (nx - 1) + (int64_t)row * nx + ix,
                   t == 0 ? 1 : 0, 1.0);
        }
    } else {
        // line order: output c = t*ny + k (t along the wall, k wall-normal); natural k*nx + t
        const int t = c / ny, k = c % ny;
        *nat = k * nx + t;
        const int64_t nh = (int64_t)ny * (nx - 1);
        const double e = ny > 1 ? 1.0 / (double)(ny - 1) : 0.0;
        if (t > 0) set_nb(b, 0, (t - 1) * ny + k, (int64_t)k * (nx - 1) + (t - 1), 1, 1.0);
        if (t < nx - 1) set_nb(b, 1, (t + 1) * ny + k, (int64_t)k * (nx - 1) + t, 0, 1.0);
        if (k > 0) {
            const double a0 = pow(1000.0, 1.0 - (double)(k - 1) * e), a1 = pow(1000.0, 1.0 - (double)k * e);
            set_nb(b, 2, c - 1, nh + (int64_t)(k - 1) * nx + t, 1, sqrt(a0 * a1));
        }
        if (k < ny - 1) {
            const double a0 = pow(1000.0, 1.0 - (double)k * e), a1 = pow(1000.0, 1.0 - (double)(k + 1) * e);
            set_nb(b, 3, c + 1, nh + (int64_t)k * nx + t, 0, sqrt(a0 * a1));
        }
    }
}

__device__ __forceinline__ void cswap(Nbs &b, int i, int j) {
    const int ki = b.col[i] < 0 ? INT_MAX : b.col[i], kj = b.col[j] < 0 ? INT_MAX : b.col[j];
    const bool sw = kj < ki;
    const int c0 = b.col[i], d0 = b.dir[i];
    const int64_t f0 = b.face[i];
    const double s0 = b.scale[i];
    b.col[i] = sw ? b.col[j] : c0;
    b.face[i] = sw ? b.face[j] : f0;
    b.dir[i] = sw ? b.dir[j] : d0;
    b.scale[i] = sw ? b.scale[j] : s0;
    b.col[j] = sw ? c0 : b.col[j];
    b.face[j] = sw ? f0 : b.face[j];
    b.dir[j] = sw ? d0 : b.dir[j];
    b.scale[j] = sw ? s0 : b.scale[j];
}

template <int KIND>
__global__ void k_gen_rowlen(int nx, int ny, uint64_t seed, int n, int64_t *len) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Nbs b;
    int nat;
    neighbours<KIND>(nx, ny, key(seed, S_SPLIT), c, &nat, b);
    int m = 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) m += b.col[q] >= 0;
    len[c] = m;
}

// One quad per row; lane r writes row r of every block of the row.
template <int KIND>
__global__ __launch_bounds__(WG) void k_gen_fill(int nx, int ny, double cfl, uint64_t seed, int n,
                                                 const int32_t *__restrict__ rowptr, int32_t *__restrict__ colidx,
                                                 double *__restrict__ A, double *__restrict__ b) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    const int r = threadIdx.x & 3;
    if (c >= n) return;
    Nbs nb;
    int nat;
    neighbours<KIND>(nx, ny, key(seed, S_SPLIT), c, &nat, nb);
    // sorting network on the four slots (absent slots last)
    cswap(nb, 0, 1);
    cswap(nb, 2, 3);
    cswap(nb, 0, 2);
    cswap(nb, 1, 3);
    cswap(nb, 1, 2);
    const uint64_t kw = key(seed, S_FACE_W), ko = key(seed, S_OFFDIAG), kp = key(seed, S_DIAGPERT),
                   kr = key(seed, S_RHS);
    int pos = rowptr[c];
    double nrm = 0.0;
    int diag_slot = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (nb.col[q] < 0) continue;
        if (diag_slot < 0 && nb.col[q] > c) {   // the diagonal goes before the first larger column
            diag_slot = pos++;
            if (r == 0) colidx[diag_slot] = c;
        }
        const double w = __dmul_rn(uab(kw, (uint64_t)nb.face[q], 0.5, 1.5), nb.scale[q]);
        const uint64_t ctr = 2 * (uint64_t)nb.face[q] + (uint64_t)nb.dir[q];
        double v[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) v[cc] = __dmul_rn(uab(ko, ctr * 16 + (uint64_t)(r * 4 + cc), -1.0, 1.0), w);
        double *blk = A + (int64_t)pos * BB + r * 4;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) blk[cc] = v[cc];
        if (r == 0) colidx[pos] = nb.col[q];
        // induced 1-norm: max over columns of the absolute column sums (rows are spread over the quad)
        double cs[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            double x[4];
            gather_vec(fabs(v[cc]), x);
            cs[cc] = ((x[0] + x[1]) + x[2]) + x[3];
        }
        nrm += fmax(fmax(cs[0], cs[1]), fmax(cs[2], cs[3]));
        ++pos;
    }
    if (diag_slot < 0) {
        diag_slot = pos;
        if (r == 0) colidx[diag_slot] = c;
    }
    const double shift = nrm / cfl;
    double *blk = A + (int64_t)diag_slot * BB + r * 4;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        double p = uab(kp, (uint64_t)nat * 16 + (uint64_t)(r * 4 + cc), -0.1, 0.1);
        blk[cc] = (cc == r) ? __dadd_rn(p, __dadd_rn(shift, nrm)) : p;
    }
    b[(int64_t)c * 4 + r] = uab(kr, (uint64_t)nat * 4 + r, -1.0, 1.0);
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
    return sizeof(int64_t) * (size_t)(2 * (nn + 1) + scan_tiles(nn) + 1);
}

extern "C" abilu_status abilu_gen_build(const abilu_gen_spec *spec, int32_t *d_rowptr, int32_t *d_colidx,
                                        double *d_A, double *d_b, void *d_scratch, void *stream) {
    int64_t nn, zz;
    if (!sizes_of(spec, &nn, &zz)) return ABILU_EINVAL;
    if (!d_rowptr || !d_colidx || !d_A || !d_b || !d_scratch) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)nn;
    int64_t *len = (int64_t *)d_scratch;
    int64_t *tmp = len + (nn + 1);
    int64_t *tot = tmp + (nn + 1);
    {
        ProfScope ps("gen_rowlen", s, 8.0 * nn);
        if (spec->kind == ABILU_GEN_TRI)
            k_gen_rowlen<ABILU_GEN_TRI><<<div_up(n, 256), 256, 0, s>>>(spec->nx, spec->ny, spec->seed, n, len);
        else
            k_gen_rowlen<ABILU_GEN_ANISO><<<div_up(n, 256), 256, 0, s>>>(spec->nx, spec->ny, spec->seed, n, len);
    }
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    if (!hip_ok(scan_exclusive(nn, len, tmp, tot, nullptr, d_rowptr, s), "gen rowptr scan")) return ABILU_EDEVICE;
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
