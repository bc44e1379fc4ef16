/*
 * abilu_gen.h - seeded synthetic 4x4-block Jacobians generated on the device: the input source of
 * the serving benchmark and its tests. It holds none of the preconditioner's arithmetic.
 *
 * The matrices have the structure of the paper's finite-volume Jacobians (Section 2): one 4x4
 * block row per cell, one block per face neighbour, and a diagonal shifted by the pseudo-time
 * term (local time step equation): A_ii = (sum_j ||A_ij||_1 (1 + 1/CFL)) I + P_i. Face weight
 * w_f ~ U(0.5,1.5) shared by A_ij and A_ji, block entries U(-1,1) w_f, P_i ~ U(-0.1,0.1), RHS
 * U(-1,1). Random numbers use the SplitMix64 finaliser on (seed, stream, natural index), the
 * same keys as the host generator (paper_1912_00539_amd/workloads.py), so a device-generated
 * case has the host case's pattern exactly and its values up to summation order.
 *
 *   ABILU_GEN_TRI  : nx x ny quads cut into two triangles along seeded random diagonals, cells in
 *                    natural order (quad-row-major, the two triangles of a quad adjacent)
 *   ABILU_GEN_ANISO: nx cells along a wall x ny wall-normal layers, wall-normal faces of layers
 *                    k, k+1 scaled by sqrt(AR_k AR_{k+1}), AR_k = 1000^(1 - k/(ny-1)); cells in
 *                    line order (each wall-normal line contiguous, from the wall outward)
 */
#ifndef ABILU_GEN_H
#define ABILU_GEN_H

#include <stddef.h>
#include <stdint.h>

#include "abilu.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { ABILU_GEN_TRI = 0, ABILU_GEN_ANISO = 1 } abilu_gen_kind;

typedef struct {
    int32_t kind;    /* abilu_gen_kind */
    int32_t nx, ny;  /* mesh dimensions (>= 1) */
    double cfl;      /* pseudo-time CFL number (> 0) */
    uint64_t seed;
} abilu_gen_spec;

/* Block rows N and block nonzeros Z of the case (host only, no device work). */
abilu_status abilu_gen_sizes(const abilu_gen_spec *spec, int32_t *n, int64_t *nnzb);

/* Device scratch bytes needed by abilu_gen_build. */
size_t abilu_gen_scratch_bytes(const abilu_gen_spec *spec);

/* Generate the case into caller device buffers: d_rowptr int32[N+1], d_colidx int32[Z],
 * d_A double[Z][4][4] (CSR order, row-major blocks), d_b double[4N]. Non-blocking, allocates
 * nothing (d_scratch >= abilu_gen_scratch_bytes). */
abilu_status abilu_gen_build(const abilu_gen_spec *spec, int32_t *d_rowptr, int32_t *d_colidx, double *d_A,
                             double *d_b, void *d_scratch, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ABILU_GEN_H */
