/*
 * A C program that uses libabilu through its C ABI alone (no Python, no torch): it builds a
 * seeded 4x4-block system on a 2-D grid (5-point stencil, block diagonally dominant), uploads it
 * with the HIP runtime, builds the pattern, runs one asynchronous FP32 factor sweep and FGMRES(30)
 * with 3 apply sweeps to rtol, and checks the returned x by computing ||b - A x|| / ||b|| on the
 * host. It also checks that an invalid argument comes back as an error code. Prints one line and
 * exits 0 when every check holds.
 *
 * Usage: abilu_c_solve [nx ny]
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "abilu.h"

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* uniform in [-1, 1), xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) / 4503599627370496.0 - 1.0;
}

#define CHECK_HIP(x)                                                              \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            return 2;                                                             \
        }                                                                         \
    } while (0)
#define CHECK_ABI(x)                                                              \
    do {                                                                          \
        abilu_status s_ = (x);                                                    \
        if (s_ < 0) {                                                             \
            fprintf(stderr, "abilu error %d (%s) at %s:%d\n", (int)s_, abilu_status_string(s_), __FILE__, __LINE__); \
            return 3;                                                             \
        }                                                                         \
    } while (0)

int main(int argc, char **argv) {
    const int nx = argc > 2 ? atoi(argv[1]) : 40, ny = argc > 2 ? atoi(argv[2]) : 30;
    const int n = nx * ny;
    /* pattern: the cell and its grid neighbours, columns ascending */
    int32_t *rowptr = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    int32_t *colidx = (int32_t *)malloc(sizeof(int32_t) * 5 * n);
    int z = 0;
    rowptr[0] = 0;
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const int i = iy * nx + ix;
            if (iy > 0) colidx[z++] = i - nx;
            if (ix > 0) colidx[z++] = i - 1;
            colidx[z++] = i;
            if (ix < nx - 1) colidx[z++] = i + 1;
            if (iy < ny - 1) colidx[z++] = i + nx;
            rowptr[i + 1] = z;
        }
    /* values: off-diagonal blocks uniform in [-1, 1); diagonal blocks (1 + sum of the row's
     * off-diagonal block 1-norms) I plus a small perturbation */
    double *A = (double *)malloc(sizeof(double) * 16 * (size_t)z);
    double *b = (double *)malloc(sizeof(double) * 4 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        double s = 1.0;
        int d = -1;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (colidx[e] == i) {
                d = e;
                continue;
            }
            double norm1 = 0.0;
            for (int c = 0; c < 4; ++c) {
                double col = 0.0;
                for (int r = 0; r < 4; ++r) {
                    A[16 * (size_t)e + 4 * r + c] = urand();
                    col += fabs(A[16 * (size_t)e + 4 * r + c]);
                }
                if (col > norm1) norm1 = col;
            }
            s += norm1;
        }
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) A[16 * (size_t)d + 4 * r + c] = (r == c ? s : 0.0) + 0.1 * urand();
        for (int r = 0; r < 4; ++r) b[4 * i + r] = urand();
    }

    int32_t *d_rowptr, *d_colidx;
    double *d_A, *d_b, *d_x;
    float *d_LU, *d_Dinv;
    CHECK_HIP(hipMalloc((void **)&d_rowptr, sizeof(int32_t) * (n + 1)));
    CHECK_HIP(hipMalloc((void **)&d_colidx, sizeof(int32_t) * z));
    CHECK_HIP(hipMalloc((void **)&d_A, sizeof(double) * 16 * (size_t)z));
    CHECK_HIP(hipMalloc((void **)&d_b, sizeof(double) * 4 * (size_t)n));
    CHECK_HIP(hipMalloc((void **)&d_x, sizeof(double) * 4 * (size_t)n));
    CHECK_HIP(hipMalloc((void **)&d_LU, sizeof(float) * 16 * (size_t)z));
    CHECK_HIP(hipMalloc((void **)&d_Dinv, sizeof(float) * 16 * (size_t)n));
    CHECK_HIP(hipMemcpy(d_rowptr, rowptr, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_colidx, colidx, sizeof(int32_t) * z, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_A, A, sizeof(double) * 16 * (size_t)z, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_b, b, sizeof(double) * 4 * (size_t)n, hipMemcpyHostToDevice));

    /* an invalid block size is an error code, not a crash */
    abilu_pattern *bad = NULL;
    if (abilu_build_pattern(n, d_rowptr, d_colidx, 3, NULL, &bad) != ABILU_EINVAL || bad != NULL) {
        fprintf(stderr, "block size 3 was not rejected\n");
        return 4;
    }

    abilu_pattern *p = NULL;
    CHECK_ABI(abilu_build_pattern(n, d_rowptr, d_colidx, 4, NULL, &p));
    const int restart = 30;
    const size_t wb = abilu_workspace_bytes(p, ABILU_F32, restart);
    void *d_work;
    CHECK_HIP(hipMalloc(&d_work, wb));
    CHECK_HIP(hipMemset(d_work, 0, wb));
    CHECK_ABI(abilu_factor(p, d_A, d_LU, d_Dinv, ABILU_F32, 1, ABILU_ASYNC, ABILU_INIT_FROM_A, d_work, wb, NULL));
    abilu_fgmres_result res;
    const double rtol = 1e-8;
    const abilu_status st = fgmres_solve(p, d_A, d_b, d_x, restart, 500, rtol, d_LU, d_Dinv, ABILU_F32, 3,
                                         ABILU_ASYNC, ABILU_FGMRES_ZERO_GUESS, d_work, wb, NULL, &res);
    CHECK_ABI(st);

    /* the residual of the returned x, on the host */
    double *x = (double *)malloc(sizeof(double) * 4 * (size_t)n);
    CHECK_HIP(hipMemcpy(x, d_x, sizeof(double) * 4 * (size_t)n, hipMemcpyDeviceToHost));
    double rr = 0.0, bb = 0.0;
    for (int i = 0; i < n; ++i)
        for (int r = 0; r < 4; ++r) {
            double acc = b[4 * i + r];
            for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
                for (int c = 0; c < 4; ++c) acc -= A[16 * (size_t)e + 4 * r + c] * x[4 * colidx[e] + c];
            rr += acc * acc;
            bb += b[4 * i + r] * b[4 * i + r];
        }
    const double rel = sqrt(rr / bb);
    const int ok = st == ABILU_OK && res.converged && rel <= rtol && fabs(rel - res.rel_true_residual) <= 1e-12;
    printf("%s: n=%d blocks=%d iters=%d restarts=%d rel_residual=%.3e (library %.3e)\n", ok ? "OK" : "FAIL", n, z,
           res.iters, res.restarts, rel, res.rel_true_residual);

    CHECK_ABI(abilu_pattern_destroy(p));
    hipFree(d_work);
    hipFree(d_rowptr);
    hipFree(d_colidx);
    hipFree(d_A);
    hipFree(d_b);
    hipFree(d_x);
    hipFree(d_LU);
    hipFree(d_Dinv);
    free(rowptr);
    free(colidx);
    free(A);
    free(b);
    free(x);
    return ok ? 0 : 1;
}
