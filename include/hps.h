/*
 * hps.h - C ABI of the MI355X (gfx950) RKHPS per-stage solver.
 *
 * Method: Chen, Appelo, Babb & Martinsson, "Fast and high-order approximation
 * of parabolic equations using hierarchical direct solvers and implicit
 * Runge-Kutta methods" (arXiv 2306.02526).
 *
 *   u_t = L u + q + g(u)  in (0,T) x Omega,  u = f on the boundary      (eq. 1)
 *   L u = cxx u_xx + cyy u_yy + cx u_x + cy u_y + c0 u   (eq. 3 with c12 = 0)
 *
 * Omega = [x0,x1] x [y0,y1] is split into n1 x n2 equal squares carrying p x p
 * Chebyshev nodes each; corner nodes are dropped (Sec. 2.1).  Every implicit
 * ESDIRK stage solves (I - gamma*dt*L) u_i = rhs_i (eq. 10) with the HPS
 * direct solver, built once for the fixed gamma*dt and then reused.
 *
 * Conventions for every entry point
 *   - Return value: HPS_OK (0) or a negative HPS_E* code; hps_last_error()
 *     returns a thread-local message describing the last failure.
 *   - "device" arrays are HIP device allocations (hipMalloc, or PyTorch CUDA
 *     tensors); a host pointer where a device pointer is required is rejected
 *     with HPS_EINVAL.  "host" arrays are ordinary host memory.
 *   - All arrays are owned by the caller and only read or written during the
 *     call (stream-ordered calls: until the given stream reaches that point).
 *     Handles (hps_op, ark_ctx) are owned by the library; release them with
 *     hps_free / ark_free.  One handle serves one stream at a time; calls on a
 *     handle from two streams at once race.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it; hps_build returns after the build has finished.
 *   - Canonical node order of every length-N vector (N = n_int + n_edge):
 *       1. leaf interiors: leaf (i, j) in order j*n1 + i, then its (p-2)^2
 *          interior nodes row-major with x fastest;
 *       2. vertical edges: grid line k = 0..n1, leaf row j, node ascending in y;
 *       3. horizontal edges: grid line k = 0..n2, leaf column i, node
 *          ascending in x.
 *     Local Chebyshev nodes on a leaf [a, a+h] are a + h (1 - cos(m pi/(p-1)))/2.
 *     n_int = n1 n2 (p-2)^2, n_edge = (p-2)(2 n1 n2 + n1 + n2)  (Sec. 2.1).
 *     "boundary" vectors (length n_bdry = 2 (p-2)(n1+n2)) list the edge nodes on
 *     the outer boundary in canonical order; "interface" vectors (length
 *     n_iface = n_edge - n_bdry) list the remaining edge nodes in canonical order.
 */
#ifndef HPS_MI355X_H
#define HPS_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HPS_API __attribute__((visibility("default")))

#define HPS_OK              0
#define HPS_EINVAL         -1   /* invalid argument (sizes, pointers, flags)        */
#define HPS_ENOMEM         -2   /* device allocation failed                          */
#define HPS_EDEVICE        -3   /* HIP runtime or kernel launch error                */
#define HPS_ESINGULAR      -4   /* zero pivot while building an inverse              */
#define HPS_ENOTCONVERGED  -5   /* iterative refinement did not reach its tolerance  */
#define HPS_EBUSY          -6   /* a bounded queue is full (srv_submit); retry later */

/* hps_build flags */
#define HPS_FP64     0   /* stored operators and their application in FP64.  With at
                            least two tree levels, the level sweeps of an operator
                            without HPS_WIDE_TILES (FP64, complex, or FP32_IR: FP32
                            copies for the FP32 passes) go through composite operators
                            of level pairs built with it: the two levels'
                            products multiplied out once per node of the upper level,
                            one launch per pair and direction instead of one per
                            level, for about 1.4 times the level operators' memory.
                            The environment variable HPS_COMPOSE=0 at build time turns
                            them off (HPS_COMPOSE=1 forces them where the tuner chose
                            against them); results differ by rounding only.  A small
                            FP64 tree (the matrix below at most 2 MiB) also gets its
                            whole sweep without Dirichlet or jump data as one product:
                            interface values = M h_leaf, M taken at build time from the
                            operator's own sweeps of unit vectors (HPS_DIRECT=0 at build
                            time turns it off; results differ by rounding only).    */
#define HPS_FP32_IR  1   /* FP64 build; operators applied in FP32 inside an FP64
                            iterative-refinement loop (residual in FP64): corrections
                            until ||delta||_inf <= 1e-11 ||u||_inf, at most 10; a solve
                            that does not get there is redone with the FP64 operators,
                            which the operator keeps (unless HPS_IR_STRICT)          */
#define HPS_WIDE_TILES 2 /* or-ed with either: cut each tree level's operators into few
                            large row tiles (fewer workgroups per level).  For
                            operators stepped many at a time (ark_step_batched, the
                            server) and for two-component steps (ark_step_burgers);
                            one scalar problem runs at the same speed either way.   */
#define HPS_IR_STRICT 8   /* or-ed with HPS_FP32_IR: a refinement that does not reach
                            its tolerance is an error (HPS_ENOTCONVERGED) instead of
                            being redone with the FP64 operators                    */
#define HPS_TEST_FP32_SKEW 16 /* or-ed with HPS_FP32_IR, for tests of the refinement's
                            failure handling only: the FP32 copy of every leaf inverse
                            is stored multiplied by 1.5, so each correction removes only
                            about half of the error and refinement cannot converge   */
#define HPS_AUTOTUNE 32  /* or-ed with the others (not with HPS_WIDE_TILES): choose how finely
                            every tree level's products are cut into workgroups by timing
                            the candidates on the device: the first build of an operator
                            class (grid shape, p, precision, real/complex, uniform
                            coefficients) builds it with each candidate tiling and times
                            hps_solve; the choice is kept for the process and, when the
                            environment variable HPS_TUNE_FILE names a file, read from and
                            written to it (JSON: class -> chosen minimum of workgroups per
                            level and the measured microseconds per solve).  Results differ
                            from untuned ones by rounding only.                        */
#define HPS_UNIFORM_COEFFS 4 /* or-ed with the above: the caller states that every
                            coefficient of L is the same at every node (e.g. L = eps
                            Lap).  Then every leaf, and every node of one tree level,
                            has the same operators: they are computed and stored
                            once (one leaf, one node per level) and all workgroups
                            read that copy, which stays in the on-chip caches
                            (operator memory / number of leaves, and far less HBM
                            traffic).  hps_build checks the claim (HPS_EINVAL if
                            any coefficient varies); results are bitwise those of
                            the build without the flag.                             */

typedef struct {
    double x0, x1, y0, y1;   /* domain; (x1-x0)/n1 must equal (y1-y0)/n2 (square leaves) */
    int32_t n1, n2;          /* leaves per direction, powers of two, n1*n2 <= 2^14      */
    int32_t p;               /* Chebyshev nodes per leaf side, 3 <= p <= 24             */
} hps_grid;

/* Coefficients of L sampled at the n_int interior nodes (canonical order);
 * device arrays.  A NULL member means that coefficient is zero. */
typedef struct {
    const double *cxx, *cyy, *cx, *cy, *c0;
} hps_coeffs;

typedef struct {
    int32_t ir_iterations;    /* FP32_IR: correction solves used by the last call       */
    double  last_correction;  /* FP32_IR: ||delta||_inf / ||u||_inf of the last one     */
    int32_t fp64_fallbacks;   /* FP32_IR: solves of the last call that did not converge
                                 and were redone with the FP64 operators                */
} hps_info;

typedef struct hps_op  hps_op;
typedef struct ark_ctx ark_ctx;

/* Thread-local text of the last error (never NULL). */
HPS_API const char *hps_last_error(void);

/* Node counts of a grid (Sec. 2.1).  Returns N, or a negative error code.
 * n_int / n_iface / n_bdry may be NULL. */
HPS_API int64_t hps_num_nodes(const hps_grid *grid, int64_t *n_int, int64_t *n_iface, int64_t *n_bdry);

/* Coordinates of the N nodes in canonical order; x, y are host arrays of N. */
HPS_API int hps_nodes(const hps_grid *grid, double *x, double *y);

/* Build the HPS solver for A = I - gamma_dt * L (eq. 10): leaf operators
 * S = -A_ii^{-1} A_ib and DtN maps T (eqs. 5-6), then the merges
 * S_tau = (T^a_33 - T^b_33)^{-1} [-T^a_31 | T^b_32] and
 * T_tau = diag(T^a_11, T^b_22) + [T^a_13; T^b_23] S_tau up the tree (Sec. 2.1),
 * all on the GPU in FP64.  gamma_dt > 0.  coeffs: device arrays (see above).
 * Returns HPS_ESINGULAR if a pivot vanishes.  *out receives the handle. */
HPS_API int hps_build(const hps_grid *grid, const hps_coeffs *coeffs, double gamma_dt, int flags,
              void *stream, hps_op **out);

/* The same for complex coefficients (the regularised NLS of Sec. 5.5 has L = (a eps + i)
 * Lap): re and im hold the real and imaginary parts of each coefficient (device arrays,
 * NULL members zero).  The operator is the real embedding [[Re, -Im], [Im, Re]] of the
 * complex one, built and applied in FP64; every complex vector the operator takes or
 * returns (hps_solve, ark_step) is two planes of the real layout, real part then
 * imaginary part (body [2][n_int], u [2][N], dirichlet [2][n_bdry], jump [2][n_iface],
 * per right-hand side).  flags: HPS_FP64, optionally HPS_WIDE_TILES and
 * HPS_UNIFORM_COEFFS (not HPS_FP32_IR); p <= 18 (one leaf's embedded operator fills a
 * workgroup tile).  Stored operators take about 4x the real ones. */
HPS_API int hps_build_complex(const hps_grid *grid, const hps_coeffs *re, const hps_coeffs *im, double gamma_dt,
                              int flags, void *stream, hps_op **out);

/* Bytes of device memory held by the operator (stored operators + workspace). */
HPS_API int64_t hps_op_bytes(const hps_op *op, int64_t *operator_bytes);

/* Solve A u = body at interior nodes, u = dirichlet on the outer boundary and
 * flux_alpha - flux_beta = jump on interface edge nodes (alpha the left/bottom
 * leaf; flux in the coordinate direction), for nrhs right-hand sides:
 * Algorithm 1 of Sec. 2.1 with the body load and jump added to the sweeps.
 *   body      device [nrhs][n_int]
 *   dirichlet device [nrhs][n_bdry] or NULL (zero)
 *   jump      device [nrhs][n_iface] or NULL (zero)
 *   u         device [nrhs][N] (output, canonical order)
 * info may be NULL; when given, the call waits for the stream to finish. */
HPS_API int hps_solve(hps_op *op, int nrhs, const double *body, const double *dirichlet,
              const double *jump, double *u, void *stream, hps_info *info);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hps_solve without allocation.
 * Same arguments, layouts and results as hps_solve (bitwise: the same kernels in the
 * same order), without `info`, for real operators built with HPS_FP64 (HPS_WIDE_TILES
 * and HPS_UNIFORM_COEFFS allowed); FP32_IR and complex operators give HPS_EINVAL.
 * The solve's intermediate data (leaf and level boundary values, particular solutions
 * and fluxes, split-K partials) go to one fixed device array of
 * HPS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends (64 x 64 leaves at p = 16 use 19.1 MiB of it); an operator whose solve
 * needs more is rejected with HPS_EINVAL.  Nothing is allocated: the first call on a
 * device only looks up the array's address.  The array is shared by every call on that
 * GPU and keeps the last call's contents (the call clears what must start at zero), so
 * calls that overlap on one GPU (two streams or two threads at once) race: serialize
 * them.  Stream-ordered; returns without waiting. */
#define HPS_NOALLOC_SCRATCH_BYTES (32LL << 20)
HPS_API int hps_solve_noalloc(hps_op *op, int nrhs, const double *body, const double *dirichlet,
                              const double *jump, double *u, void *stream);

HPS_API void hps_free(hps_op *op);

/* Kernel timing for measurement tools: while enabled, every kernel family launched
 * for this operator (leaf_up, level_up, level_down, leaf_down, eval, residual,
 * update; per precision) is bracketed by HIP events on its launch stream. */
HPS_API int hps_profile_enable(hps_op *op, int enable);

/* Aggregate the recorded events per kernel family and clear them.  Writes up to
 * max entries (static name, number of launches, total milliseconds) into the
 * host arrays names / launches / total_ms (each may be NULL) and returns the
 * number of families seen.  Waits for the recorded events to complete. */
HPS_API int hps_profile_read(hps_op *op, int max, const char **names, int64_t *launches, double *total_ms);

/* Additive Runge-Kutta tableau (Sec. 3.1, Table 1): ESDIRK (A, b, c) with
 * A[0][0] = 0 and A[i][i] = gamma for i >= 1, ERK (Ahat, bhat, c), row-major
 * s x s host arrays, 2 <= s <= 8. */
typedef struct {
    int32_t s;
    const double *A, *b, *c, *Ahat, *bhat;
} ark_tableau;

/* Explicit nonlinearity g(u) = g0 + g1 u + g2 u^2 + g3 u^3 (kind = 1), or none (kind = 0).
 * For a complex operator: kind = 2, g(u) = (g0 + i g1) u + (g2 + i g3) |u|^2 u (the NLS of
 * Sec. 5.5 has g0 = b eps, g1 = 0, g2 = -c eps, g3 = 1), or kind = 0. */
typedef struct {
    int32_t kind;
    double g0, g1, g2, g3;
} ark_g;

/* Time-stepping context for the stage formulation (eqs. 9-11) on a built
 * operator.  Requires |A[1][1]*dt - gamma_dt| <= 1e-14 |gamma_dt|; g may be NULL. */
HPS_API int ark_create(hps_op *op, const ark_tableau *tab, double dt, const ark_g *g, ark_ctx **out);

/* One step t -> t + dt of the stage formulation, in place on u (device [N]):
 *   stage 1: L u^n and F_1 = q(t) + g(u^n);
 *   stages i = 2..s: solve (I - gamma dt L) u_i = u^n + dt sum_{j<i} a_ij L u_j
 *                    + dt sum_{j<i} ahat_ij F_j with u_i = f(t + c_i dt) on the
 *                    boundary, then L u_i and F_i = q(t + c_i dt) + g(u_i);
 *   completion:      interior u^{n+1} = u^n + dt sum_j (b_j L u_j + bhat_j F_j),
 *                    boundary f(t + dt), interface nodes from flux continuity.
 * Source q, by one of (or none: q = 0):
 *   q_stages  device [s][n_int]: q at t + c_i dt;
 *   q_space   device [n_int] with q_time host [s]: q = q_time[i] * q_space.
 * f_stages: device [s+1][n_bdry], f at t + c_i dt (i < s) and at t + dt; NULL = 0.
 * Complex operator (hps_build_complex): u device [2][N], f_stages [s+1][2][n_bdry], no
 * source (q_stages and q_space must be NULL; HPS_EINVAL otherwise). */
HPS_API int ark_step(ark_ctx *ctx, double t, double *u, const double *q_stages,
             const double *q_space, const double *q_time, const double *f_stages, void *stream);

/* One step t -> t + dt of the slope formulation (Sec. 3.1) with the flux-jump
 * penalisation of Sec. 3.1, in place on u (device [N]):
 *   k_1 = L u^n + q(t),  l_1 = g(u^n);
 *   (I - gamma dt L) k_i = L u^n + dt sum_{j<i} (a_ij L k_j + ahat_ij L l_j) + q(t + c_i dt),
 *   l_i = g(u^n + dt sum_{j<=i} a_ij k_j + dt sum_{j<i} ahat_ij l_j),        i = 2..s;
 *   u^{n+1} = u^n + dt sum_j (b_j k_j + bhat_j l_j) at every node.
 * k_i on the outer boundary = fdot_stages[i] (device [s][n_bdry]: the time derivative of
 * the Dirichlet data at t + c_i dt; NULL = 0); l_i = 0 there, so with g the Dirichlet data
 * must not depend on time.  Every k_i takes the flux jump -(flux_alpha - flux_beta)(u^n)/dt
 * across the interfaces (the penalised condition), so u^{n+1} is flux-continuous when
 * g = 0.  k_1 and l_i are explicit: interface values of k_1 come from that condition,
 * l_i is pointwise.  q as in ark_step.  The first call allocates the slopes' workspace
 * (about 2 s (N + n_int) doubles with g, half without). */
HPS_API int ark_step_slope(ark_ctx *ctx, double t, double *u, const double *q_stages,
                           const double *q_space, const double *q_time, const double *fdot_stages,
                           void *stream);

/* One step t -> t + dt of the two-dimensional viscous Burgers system of Sec. 5.4,
 *   u_t = L u - (u u_x + v u_y),   v_t = L v - (u v_x + v v_y),
 * (L = eps Lap there; any operator built by hps_build is accepted), in the stage
 * formulation (eqs. 9-11) for both components, in place on u and v (device [N] each,
 * different arrays).  cu and cv are the contexts of the two components: created by
 * ark_create on the same FP64 operator (HPS_FP32_IR is rejected) with the same tableau
 * and dt and with g = NULL (the advection terms are the explicit part; they couple the
 * components at every stage and are evaluated by collocation on the leaves, like L).
 * Each stage solves both components' systems together: every operator block is read
 * once for the two right-hand sides.
 * fu_stages, fv_stages: device [s+1][n_bdry], the Dirichlet data of u and v at
 * t + c_i dt (i < s) and at t + dt; NULL = 0.  The first call allocates solve buffers
 * for cv (about the operator's workspace, O(N) doubles).
 * Errors: HPS_EINVAL for NULL or mismatched handles, equal u and v, or an FP32_IR
 * operator; HPS_EDEVICE for a failed launch. */
HPS_API int ark_step_burgers(ark_ctx *cu, ark_ctx *cv, double t, double *u, double *v,
                             const double *fu_stages, const double *fv_stages, void *stream);

/* Refinement record of the last ark_step on an FP32_IR operator: ir_iterations = the
 * corrections per stage solve (the most any stage used), last_correction = the largest
 * final ||delta||_inf / ||u||_inf over the stages, fp64_fallbacks = stages redone with the
 * FP64 operators.  Zeros for FP64 operators.
 * An FP32_IR ark_step of the stage formulation is replayed from a captured HIP graph with
 * a fixed number of corrections per stage (the most the first, host-checked, step needed);
 * after the replay the call waits for the stream and reads every stage's last correction
 * norm: if one missed the tolerance, the step is redone from the saved u^n with
 * host-checked refinement and FP64 re-solves where needed (HPS_IR_STRICT: HPS_ENOTCONVERGED
 * instead, u then holds the unconverged step), and later steps use more corrections. */
HPS_API int ark_info(const ark_ctx *ctx, hps_info *info);

/* Number of implicit stage solves performed per ark_step (s - 1). */
HPS_API int ark_stage_solves_per_step(const ark_ctx *ctx);

HPS_API void ark_free(ark_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* HPS_MI355X_H */
