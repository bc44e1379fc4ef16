/*
 * abilu_serve.h - continuous batching of independent preconditioned FGMRES solves on one GPU.
 *
 * Each request is one linear system of the kind the paper solves once per pseudo-time step
 * (Section 2: a 4x4-block Jacobian with the local-time-step diagonal shift), generated on the
 * device from an abilu_gen_spec (abilu_gen.h), preconditioned by block ILU(0) sweeps (Section 4:
 * factor sweeps, then Jacobi sweeps on the triangular factors, Algorithm 5) and solved by
 * restarted FGMRES from a zero initial guess, exactly as fgmres_solve does for one system.
 *
 * The server owns no request memory: the caller hands it one device pool at creation. A request
 * is admitted, in arrival order, when a slot is free and its footprint (abilu_serve_footprint:
 * the system in FP64, factor and inverse diagonal blocks in the preconditioner precision, the
 * FGMRES bases V and Z in FP64, pattern arrays) fits in the pool; it holds that block until it
 * finishes. Every tick advances every admitted request by one step of its own solve (its factor
 * and initial residual, one Arnoldi step, or the end of a restart cycle); requests in the same
 * step run in one batched launch per kernel, each workgroup working on one tile of one request.
 * Admission (device generation and pattern analysis) runs on a second stream and overlaps the
 * ticks. A request's arithmetic never depends on the other requests: its tiles, reductions and
 * stopping decisions are those it would have alone (in ABILU_SYNC mode the result is bitwise the
 * same alone, in any mix, and as from abilu_factor + fgmres_solve; ABILU_ASYNC sweeps update in
 * place, so their rounding depends on scheduling as in the single-system path).
 *
 * Errors: entry points return abilu_status; a failed request records its status in its result
 * (ABILU_ENOMEM: larger than the whole pool, ABILU_EPATTERN: invalid generated pattern,
 * ABILU_EINVAL: invalid spec) without stopping the others. ABILU_EDEVICE from a step means a
 * HIP call failed; the server must then be destroyed. Calls on one server must not overlap.
 */
#ifndef ABILU_SERVE_H
#define ABILU_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "abilu.h"
#include "abilu_gen.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct abilu_server abilu_server;

typedef struct {
    int32_t prec;           /* abilu_prec of the preconditioner (factor, sweeps) */
    int32_t mode;           /* abilu_mode of the factor and apply sweeps */
    int32_t factor_sweeps;  /* >= 0; 0 = ILU(0) initial guess X = A only */
    int32_t apply_sweeps;   /* >= 0; 0 = no preconditioner */
    int32_t restart;        /* FGMRES(m), 1 <= m <= 256 */
    int32_t maxit;          /* >= 0, Arnoldi steps in total */
    double rtol;            /* stop when ||b - A x|| <= rtol ||b|| (true residual, cycle end) */
    int32_t max_active;     /* admitted requests at most (1..4096); 1 = one solve at a time */
    int32_t reserved;       /* 0 */
} abilu_serve_config;

typedef struct {
    abilu_gen_spec gen;     /* the system to solve */
    double arrival_s;       /* abilu_serve_run: release time in seconds after the run starts;
                               abilu_serve_submit: ignored (released at once) */
    double *d_x_out;        /* optional device buffer double[4N] that receives the solution */
} abilu_request;

typedef struct {
    int32_t status;             /* abilu_status of the solve (OK, WARN_*, ENONFINITE, E*) */
    int32_t n;                  /* block rows */
    int64_t nnzb;               /* block nonzeros */
    int32_t iters, restarts, converged, reorth;
    uint32_t flags;             /* ABILU_FLAG_* of the factor */
    int32_t reserved;
    double rel_true_residual;   /* ||b - A x|| / ||b|| at the end */
    double t_arrival, t_admit, t_done;  /* seconds on the server's clock */
    int64_t footprint_bytes;    /* pool bytes the request held */
} abilu_request_result;

/* Pool bytes a request of this spec holds under this configuration (host only). 0 if invalid. */
size_t abilu_serve_footprint(const abilu_serve_config *cfg, const abilu_gen_spec *spec);

/* Create a server on the current device. d_pool: caller device memory of pool_bytes (256-byte
 * aligned), used for nothing else while the server lives; the caller frees it after destroy. */
abilu_status abilu_serve_create(const abilu_serve_config *cfg, void *d_pool, size_t pool_bytes,
                                abilu_server **out);
abilu_status abilu_serve_destroy(abilu_server *srv);

/* Queue a request (released now); *id identifies it for abilu_serve_poll. */
abilu_status abilu_serve_submit(abilu_server *srv, const abilu_request *req, int64_t *id);

/* One tick on `stream`: admit what fits, advance every admitted request by one step, retire the
 * finished ones. Blocking (waits for the tick). *active / *queued (optional) receive the counts
 * after the tick. */
abilu_status abilu_serve_step(abilu_server *srv, void *stream, int32_t *active, int32_t *queued);

/* *done = 1 and *out filled once request `id` has finished (its x copied to d_x_out). */
abilu_status abilu_serve_poll(abilu_server *srv, int64_t id, int32_t *done, abilu_request_result *out);

/* Serve a whole request trace: request q is released arrival_s seconds after the call starts;
 * returns when all have finished. results[q] as from abilu_serve_poll; *elapsed_s (optional)
 * receives the wall time of the run. */
abilu_status abilu_serve_run(abilu_server *srv, const abilu_request *reqs, int32_t count,
                             abilu_request_result *results, double *elapsed_s, void *stream);

typedef struct {
    int64_t ticks;      /* ticks that launched work */
    int64_t launches;   /* batched kernel launches */
    int64_t admitted;   /* requests admitted (generated and analysed) */
    int64_t retired;    /* requests finished after at least one tick */
    double bytes;       /* algorithmic bytes of the batched solve kernels: for every launch, the
                           sum over its members of what the single-system kernel touches (every
                           array element once); generation and pattern analysis not included */
} abilu_serve_stats_t;

/* Counters since the server was created (host only). */
abilu_status abilu_serve_stats(const abilu_server *srv, abilu_serve_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* ABILU_SERVE_H */
