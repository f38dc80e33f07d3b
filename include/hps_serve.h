/*
 * hps_serve.h - a time-stepping server over the handles of hps.h.
 *
 * Jobs are whole time integrations: `steps` steps of the stage formulation
 * (Sec. 3.1, eqs. 9-11; ark_step in hps.h) of one problem.  A server owns a
 * thread on the device that was current at srv_create, and
 *   - an operator cache: the HPS operator of (grid, coefficient key, gamma*dt,
 *     flags) is built once (hps_build, with HPS_WIDE_TILES added to the job's
 *     flags) and shared by every job with that key;
 *     unreferenced operators are evicted least-recently-used first when a build
 *     would exceed the cache budget;
 *   - admission: jobs are admitted first-come first-served while fewer than
 *     max_active jobs run and their device memory fits in the budget: the operator
 *     (when not cached) and the job's stepping context (its stage vectors L u_j, F_j,
 *     its solve buffers and, for FP32_IR, its refinement vectors).  Contexts of
 *     finished jobs are kept for later jobs of the same operator (at most four per
 *     operator) and stay charged to the budget until they are reused or freed; to make
 *     room, kept contexts are freed first, then unreferenced operators.  A job that
 *     does not fit waits (in arrival order) until running jobs release memory; one
 *     that could never fit fails with HPS_ENOMEM;
 *   - continuous batching: every iteration advances each running job by one step
 *     in a single ark_step_batched call (include/hps_batch.h), so jobs join and
 *     leave between steps and small problems overlap on the GPU.
 * Each job runs exactly the kernels ark_step runs for it alone on that operator, in
 * the same order, so a job's result does not depend on what else the server is running.
 *
 * Arrays handed to srv_submit (coefficients, u, q_space) are caller-owned device
 * arrays and must stay valid until srv_poll reports the job finished
 * (SRV_DONE or SRV_FAILED); the server reads and writes them only in between.
 * Times in srv_status are seconds since srv_create, on the host's steady clock.
 */
#ifndef HPS_MI355X_SERVE_H
#define HPS_MI355X_SERVE_H

#include "hps.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srv_server srv_server;

typedef struct {
    int64_t cache_bytes;   /* device bytes the cached operators may hold; 0 = 3/4 of the
                              device memory free at srv_create                           */
    int32_t max_active;    /* jobs stepped together; 0 = 64, at most 4096                 */
    int32_t max_queued;    /* jobs waiting for admission at most; srv_submit returns
                              HPS_EBUSY (nothing queued) while that many wait; 0 = no
                              bound                                                       */
} srv_config;

typedef struct {
    hps_grid grid;
    uint64_t coef_key;     /* caller's name of the coefficient field: jobs with equal
                              (grid, coef_key, gamma_dt, flags) share one operator        */
    hps_coeffs coeffs;     /* device arrays of L's coefficients (read when the operator
                              of this key is not cached)                                  */
    int32_t flags;         /* HPS_FP64 or HPS_FP32_IR, optionally | HPS_UNIFORM_COEFFS     */
    ark_tableau tab;       /* copied at submission; host arrays                           */
    double dt;             /* gamma_dt of the operator = tab.A[1][1] * dt                 */
    ark_g g;               /* nonlinearity (kind 0 = none)                                */
    double t0;             /* start time                                                  */
    int32_t steps;         /* number of steps, >= 1                                       */
    double *u;             /* device [N]: initial data in, solution at t0 + steps dt out  */
    const double *q_space; /* device [n_int] or NULL: source q = q_time(t) * q_space with */
    double q_amp, q_rate;  /*   q_time(t) = q_amp * exp(q_rate * t)                       */
} srv_job;

#define SRV_QUEUED  0
#define SRV_ACTIVE  1
#define SRV_DONE    2
#define SRV_FAILED  3

typedef struct {
    int32_t state;          /* SRV_*                                                     */
    int32_t error;          /* HPS_E* code when SRV_FAILED                               */
    int32_t steps_done;
    int32_t cache_hit;      /* 1 if the job's operator was already cached when admitted */
    double submit_s, start_s, finish_s;   /* finish_s: the last step has completed     */
} srv_status;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t builds, cache_hits, evictions;
    int64_t cached_ops, cached_bytes;   /* operators held and their bytes              */
    int64_t iterations;     /* batched step calls made                                  */
    int64_t job_steps;      /* job steps taken                                          */
    int64_t context_bytes;  /* bytes charged for stepping contexts (running and kept)  */
    int64_t waits;          /* times the head of the queue waited for memory           */
} srv_stats;

/* Start a server on the current device.  cfg may be NULL (defaults). */
HPS_API int srv_create(const srv_config *cfg, srv_server **out);

/* Queue a job; *id receives its id (>= 0).  `stream` is the stream the caller
 * used to prepare the job's arrays: the job's first step waits for the work
 * enqueued on it so far.  Checks the arguments (HPS_EINVAL) before queuing;
 * HPS_EBUSY when cfg.max_queued jobs are already waiting for admission (the job is
 * not queued and the caller's arrays are not retained). */
HPS_API int srv_submit(srv_server *srv, const srv_job *job, void *stream, int64_t *id);

/* Current status of job id (HPS_EINVAL for an unknown id). */
HPS_API int srv_poll(srv_server *srv, int64_t id, srv_status *status);

/* Block until job id has finished, then report its status. */
HPS_API int srv_wait(srv_server *srv, int64_t id, srv_status *status);

/* Forget a finished job (its status is no longer kept). */
HPS_API int srv_release(srv_server *srv, int64_t id);

HPS_API int srv_get_stats(srv_server *srv, srv_stats *stats);

/* Finish every queued and running job, stop the thread, free the cache. */
HPS_API void srv_destroy(srv_server *srv);

#ifdef __cplusplus
}
#endif

#endif
