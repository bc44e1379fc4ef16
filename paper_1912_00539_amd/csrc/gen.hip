// Seeded synthetic 4x4-block Jacobians generated on the device (the serving benchmark's input
// source). Structure and random keys follow the host generator; no preconditioner arithmetic.
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

struct Nb {
    int col;      // neighbour cell (output numbering)
    int64_t face; // natural face index
    int dir;      // 0: this cell is the face's first cell (counter 2f), 1: second (2f + 1)
    double scale; // face weight factor (anisotropy)
};

// Neighbours of output row c. Returns the count (<= 4).
__device__ int neighbours(int kind, int nx, int ny, uint64_t ksplit, int c, int *nat, Nb (&nb)[4]) {
    int m = 0;
    if (kind == ABILU_GEN_TRI) {
        // natural order: cell 2q + t, quad q = iy*nx + ix
        const int q = c >> 1, t = c & 1, ix = q % nx, iy = q / nx;
        const int64_t nq = (int64_t)nx * ny;
        auto diag = [&](int qq) { return u01(ksplit, (uint64_t)qq) < 0.5; };   // '\' diagonal
        auto right_owner = [&](int qq) { return diag(qq) ? 2 * qq + 1 : 2 * qq; };
        auto left_owner = [&](int qq) { return diag(qq) ? 2 * qq : 2 * qq + 1; };
        const bool dq = diag(q);
        *nat = c;
        // diagonal face q: first cell 2q, second 2q+1
        nb[m++] = Nb{t == 0 ? 2 * q + 1 : 2 * q, (int64_t)q, t, 1.0};
        if (t == 0) {
            if (iy > 0) nb[m++] = Nb{2 * (q - nx) + 1, nq + (int64_t)ny * (nx - 1) + (int64_t)(iy - 1) * nx + ix, 1, 1.0};
            if (dq) {       // lower-left: left edge, face with quad (ix-1, iy) whose right owner is first
                if (ix > 0) nb[m++] = Nb{right_owner(q - 1), nq + (int64_t)iy * (nx - 1) + (ix - 1), 1, 1.0};
            } else {        // lower-right: right edge, first cell of face (ix, iy)-(ix+1, iy)
                if (ix < nx - 1) nb[m++] = Nb{left_owner(q + 1), nq + (int64_t)iy * (nx - 1) + ix, 0, 1.0};
            }
        } else {
            if (iy < ny - 1) nb[m++] = Nb{2 * (q + nx), nq + (int64_t)ny * (nx - 1) + (int64_t)iy * nx + ix, 0, 1.0};
            if (dq) {       // upper-right: right edge
                if (ix < nx - 1) nb[m++] = Nb{left_owner(q + 1), nq + (int64_t)iy * (nx - 1) + ix, 0, 1.0};
            } else {        // upper-left: left edge
                if (ix > 0) nb[m++] = Nb{right_owner(q - 1), nq + (int64_t)iy * (nx - 1) + (ix - 1), 1, 1.0};
            }
        }
    } else {
        // line order: output c = t*ny + k (t along the wall, k wall-normal); natural k*nx + t
        const int t = c / ny, k = c % ny;
        *nat = k * nx + t;
        auto ar = [&](int kk) { return ny > 1 ? pow(1000.0, 1.0 - (double)kk / (double)(ny - 1)) : 1000.0; };
        const int64_t nh = (int64_t)ny * (nx - 1);
        if (t > 0) nb[m++] = Nb{(t - 1) * ny + k, (int64_t)k * (nx - 1) + (t - 1), 1, 1.0};
        if (t < nx - 1) nb[m++] = Nb{(t + 1) * ny + k, (int64_t)k * (nx - 1) + t, 0, 1.0};
        if (k > 0) nb[m++] = Nb{c - 1, nh + (int64_t)(k - 1) * nx + t, 1, sqrt(ar(k - 1) * ar(k))};
        if (k < ny - 1) nb[m++] = Nb{c + 1, nh + (int64_t)k * nx + t, 0, sqrt(ar(k) * ar(k + 1))};
    }
    return m;
}

__global__ void k_gen_rowlen(int kind, int nx, int ny, uint64_t seed, int n, int64_t *len) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Nb nb[4];
    int nat;
    len[c] = 1 + neighbours(kind, nx, ny, key(seed, S_SPLIT), c, &nat, nb);
}

// One quad per row; lane r writes row r of every block of the row.
__global__ __launch_bounds__(WG) void k_gen_fill(int kind, int nx, int ny, double cfl, uint64_t seed, int n,
                                                 const int32_t *__restrict__ rowptr, int32_t *__restrict__ colidx,
                                                 double *__restrict__ A, double *__restrict__ b) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    const int r = threadIdx.x & 3;
    if (c >= n) return;
    Nb nb[4];
    int nat;
    const int m = neighbours(kind, nx, ny, key(seed, S_SPLIT), c, &nat, nb);
    // sort neighbours by column (at most 4)
    for (int a = 1; a < m; ++a)
        for (int q = a; q > 0 && nb[q].col < nb[q - 1].col; --q) {
            Nb t = nb[q];
            nb[q] = nb[q - 1];
            nb[q - 1] = t;
        }
    const uint64_t kw = key(seed, S_FACE_W), ko = key(seed, S_OFFDIAG), kp = key(seed, S_DIAGPERT),
                   kr = key(seed, S_RHS);
    const int b0 = rowptr[c];
    int pos = b0;
    double nrm = 0.0;
    int diag_slot = -1;
    for (int q = 0; q <= m; ++q) {
        const bool before = (q < m) && nb[q].col < c;
        if (diag_slot < 0 && !before) {   // the diagonal goes here
            diag_slot = pos++;
            if (r == 0) colidx[diag_slot] = c;
        }
        if (q == m) break;
        const double w = __dmul_rn(uab(kw, (uint64_t)nb[q].face, 0.5, 1.5), nb[q].scale);
        const uint64_t ctr = 2 * (uint64_t)nb[q].face + (uint64_t)nb[q].dir;
        double v[4];
        for (int cc = 0; cc < 4; ++cc) v[cc] = __dmul_rn(uab(ko, ctr * 16 + (uint64_t)(r * 4 + cc), -1.0, 1.0), w);
        double *blk = A + (int64_t)pos * BB + r * 4;
        for (int cc = 0; cc < 4; ++cc) blk[cc] = v[cc];
        if (r == 0) colidx[pos] = nb[q].col;
        // induced 1-norm: max over columns of the absolute column sums (rows are spread over the quad)
        double cs[4];
        for (int cc = 0; cc < 4; ++cc) {
            double x[4];
            gather_vec(fabs(v[cc]), x);
            cs[cc] = ((x[0] + x[1]) + x[2]) + x[3];
        }
        nrm += fmax(fmax(cs[0], cs[1]), fmax(cs[2], cs[3]));
        ++pos;
    }
    const double shift = nrm / cfl;
    double *blk = A + (int64_t)diag_slot * BB + r * 4;
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
        k_gen_rowlen<<<div_up(n, 256), 256, 0, s>>>(spec->kind, spec->nx, spec->ny, spec->seed, n, len);
    }
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    if (!hip_ok(scan_exclusive(nn, len, tmp, tot, nullptr, d_rowptr, s), "gen rowptr scan")) return ABILU_EDEVICE;
    {
        ProfScope ps("gen_fill", s, 4.0 * (nn + 1) + 132.0 * zz + 32.0 * nn);
        k_gen_fill<<<div_up(n, ROWS_PER_WG), WG, 0, s>>>(spec->kind, spec->nx, spec->ny, spec->cfl, spec->seed, n,
                                                         d_rowptr, d_colidx, d_A, d_b);
    }
    return launch_status();
}
