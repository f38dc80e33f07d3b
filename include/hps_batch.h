/*
 * hps_batch.h - many independent problems per call, on the handles of hps.h.
 *
 * A batch holds problems of different grids, orders p, gamma*dt and precision
 * (each with its own hps_op / ark_ctx built by hps.h).  Each problem is one
 * instance of the per-stage HPS solve of Sec. 2.1 (Algorithm 1) or of one step
 * of the stage formulation of Sec. 3.1 (eqs. 9-11).
 *
 * ark_step_batched runs a batch of real FP64 problems with equal stage counts, no boundary
 * data and at least two leaves each as grouped launches (problems that share an
 * operator get stepping workspaces of their own, allocated on first use):
 * one launch per leaf phase and per tree level covers every problem (levels are
 * aligned at the roots), so a step of the batch costs as many launches as a step of
 * its deepest problem; the argument records are built once per set of (context, u,
 * source) pointers and the step is replayed from a HIP graph while that set repeats.
 * Every other batch, and hps_solve_batched, runs each problem through the
 * single-problem entry point on a small pool of library-owned HIP streams of the
 * current device (default priority), largest operator first onto the least-loaded
 * stream, so that small latency-bound problems overlap; problems whose handles share
 * one hps_op stay on one stream, in batch order, because an operator's workspace
 * serves one solve at a time.  Either way each problem runs the kernels' arithmetic
 * of its single call, so results are bitwise those of the single calls.
 *
 * Stream semantics: the work starts after everything already enqueued on
 * `stream` and everything enqueued on `stream` afterwards waits for all of it,
 * exactly as if the problems had been enqueued on `stream` one by one.
 * FP32_IR problems wait on the host once per refinement pass, as in hps_solve.
 *
 * Arrays of pointers are host arrays with one entry per problem; the arrays they
 * point to follow the conventions of hps.h (device data, caller-owned).
 * Errors: HPS_EINVAL for a NULL handle or required pointer, the error of the first
 * failing problem otherwise (hps_last_error names the problem).  On an error,
 * problems already enqueued still run and `stream` still waits for them.
 */
#ifndef HPS_MI355X_BATCH_H
#define HPS_MI355X_BATCH_H

#include "hps.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Maximum number of problems per batched call. */
#define HPS_BATCH_MAX 65536

/* hps_solve for nprob problems, one right-hand side each:
 *   ops[b]        built operator of problem b
 *   body[b]       device [n_int(b)]
 *   dirichlet     NULL, or dirichlet[b] device [n_bdry(b)] or NULL (zero)
 *   jump          NULL, or jump[b] device [n_iface(b)] or NULL (zero)
 *   u[b]          device [N(b)] (output)
 *   info          NULL, or host hps_info[nprob]; when given the call waits for
 *                 every problem to finish. */
HPS_API int hps_solve_batched(hps_op *const *ops, int nprob, const double *const *body,
                              const double *const *dirichlet, const double *const *jump,
                              double *const *u, void *stream, hps_info *info);

/* ark_step for nprob problems:
 *   ctx[b]        context of problem b (ark_create)
 *   t             host [nprob], the time of each problem
 *   u[b]          device [N(b)], advanced in place from t[b] to t[b] + dt(b)
 *   q_stages, q_space, q_time, f_stages: NULL, or per-problem pointers with the
 *                 meaning they have in ark_step (q_time[b] is a host array of s). */
HPS_API int ark_step_batched(ark_ctx *const *ctx, int nprob, const double *t, double *const *u,
                             const double *const *q_stages, const double *const *q_space,
                             const double *const *q_time, const double *const *f_stages,
                             void *stream);

/* Number of library-owned streams the batch entry points spread problems over. */
HPS_API int hps_batch_streams(void);

#ifdef __cplusplus
}
#endif

#endif
