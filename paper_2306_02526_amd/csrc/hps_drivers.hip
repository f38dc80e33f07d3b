// Host drivers of the stage solve (hps_solve) and of the time step (ark_step): they only
// enqueue kernels; every arithmetic step runs on the GPU.
//
// Per FP64 ark_step (stage formulation, Sec. 3.1 eqs. 9-11, s stages):
//   leaf[eval u^n -> L u_1, F_1 | rhs_2, w, h] -> levels up -> levels down
//   leaf[u_2 -> L u_2, F_2 | rhs_3, w, h] -> levels ... -> leaf[u_s -> L u_s, F_s | u^{n+1}
//   interior, edge-flux parts] -> boundary data + interface lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hps_internal.h"

using namespace hps;

static int levels(hps_op *op, bool fp32, const double *jump, const double *dir, hipStream_t st) {
    return launch_levels(op, fp32, jump, dir, st);
}

static double ordered_bits_to_double(unsigned long long v) {
    double d;
    std::memcpy(&d, &v, sizeof(d));
    return d;
}

// One correction pass of FP64 iterative refinement around the FP32 operators:
// r = FP64 residual of the global system (interior rows rhs - (I - gamma dt L) u and the
// interface flux jumps), delta = HPS32(r) with zero boundary data, u += delta.  The pass's
// max|delta| and max|u| go to norms[0..1] (ordered bit patterns of non-negative doubles),
// folded from the leaves' values in op->ir_part.
static int ir_pass(hps_op *op, const double *rhs, const double *jump, double *u, double *norms, hipStream_t st) {
    TRY(launch_residual(op, u, rhs, jump, op->ir_r, op->ir_r3, st));
    LeafPhase up;
    up.up = LU_BODY;
    up.body = op->ir_r;
    TRY(launch_leaf(op, true, up, st));
    TRY(levels(op, true, op->n_iface ? op->ir_r3 : nullptr, nullptr, st));
    LeafPhase dn;
    dn.down = LD_IR_ADD;
    dn.u_out = u;
    dn.norm_part = op->ir_part;
    TRY(launch_leaf(op, true, dn, st));
    return launch_norm_fold(op->ir_part, (int)op->nleaves, norms, st);
}

// max|delta| / max|u| of one pass from its two ordered-bit words; converged when
// max|delta| <= IR_TOL max|u|
static bool ir_converged(const unsigned long long nb[2], double *rel) {
    const double dmax = ordered_bits_to_double(nb[0]), umax = ordered_bits_to_double(nb[1]);
    *rel = umax > 0 ? dmax / umax : dmax;
    return dmax <= IR_TOL * umax;
}

// Corrections until converged (at most IR_MAXIT), the host reading each pass's norms.
// *passes: corrections run; returns whether the last one met the tolerance.
static int ir_adaptive(hps_op *op, const double *rhs, const double *jump, double *u, hipStream_t st, int *passes,
                       double *rel, bool *ok) {
    *ok = false;
    for (int it = 1; it <= IR_MAXIT; ++it) {
        TRY(ir_pass(op, rhs, jump, u, op->ir_norms, st));
        unsigned long long nb[2];
        HPS_HIP(hipMemcpyAsync(nb, op->ir_norms, sizeof(nb), hipMemcpyDeviceToHost, st));
        HPS_HIP(hipStreamSynchronize(st));
        *passes = it;
        if (ir_converged(nb, rel)) {
            *ok = true;
            break;
        }
    }
    return HPS_OK;
}

// The FP64 solve (leaf particular solutions, level sweeps, reconstruction) of one right-hand side.
static int solve64(hps_op *op, const double *body, const double *dir, const double *jump, double *u, hipStream_t st) {
    LeafPhase up;
    up.up = LU_BODY;
    up.body = body;
    TRY(launch_leaf(op, false, up, st));
    TRY(levels(op, false, jump, dir, st));
    LeafPhase dn;
    dn.down = LD_WRITE_U;
    dn.u_out = u;
    return launch_leaf(op, false, dn, st);
}

// FP32_IR: refine the FP32 solution u of (body, dir, jump) on the host-checked loop; if it
// does not converge, redo the solve with the FP64 operators (HPS_IR_STRICT: error).
static int ir_finish(hps_op *op, const double *body, const double *dir, const double *jump, double *u,
                     hipStream_t st, hps_info *info) {
    int passes = 0;
    double rel = 0.0;
    bool ok = false;
    TRY(ir_adaptive(op, body, jump, u, st, &passes, &rel, &ok));
    if (info) {
        info->ir_iterations = std::max(info->ir_iterations, passes);
        info->last_correction = std::max(info->last_correction, rel);
    }
    if (ok) return HPS_OK;
    if (op->flags & HPS_IR_STRICT) {
        hps_set_error("iterative refinement did not converge: last correction %.3e after %d passes", rel, passes);
        return HPS_ENOTCONVERGED;
    }
    if (info) info->fp64_fallbacks += 1;
    return solve64(op, body, dir, jump, u, st);
}

// One right-hand side: leaf particular solutions, the level sweeps, reconstruction of u
// (full canonical vector), and for FP32_IR the refinement loop.
static int solve_one(hps_op *op, const double *body, const double *dir, const double *jump, double *u,
                     hipStream_t st, hps_info *inf) {
    if (op->ncomp == 2) {   // complex operator: the same sweeps on the real embedding
        LeafPhase up;
        up.up = LU_BODY;
        up.body = body;
        TRY(launch_leaf_cx(op, up, st));
        TRY(levels(op, false, jump, dir, st));
        LeafPhase dn;
        dn.down = LD_WRITE_U;
        dn.u_out = u;
        return launch_leaf_cx(op, dn, st);
    }
    const bool ir = (op->flags & HPS_FP32_IR) != 0;
    LeafPhase up;
    up.up = LU_BODY;
    up.body = body;
    TRY(launch_leaf(op, ir, up, st));
    TRY(levels(op, ir, jump, dir, st));
    LeafPhase dn;
    dn.down = LD_WRITE_U;
    dn.u_out = u;
    TRY(launch_leaf(op, ir, dn, st));
    if (ir) TRY(ir_finish(op, body, dir, jump, u, st, inf));
    return HPS_OK;
}

// Solve buffers for right-hand sides 1..n of a multi-right-hand-side solve (made once per
// operator, one allocation each).
static int multi_workspaces(hps_op *op, int n) {
    for (int k = 0; k < n; ++k) {
        if (op->mws[k]) continue;
        int64_t co = 0, cb = 0;
        const int64_t bytes = workspace_layout(op, nullptr, nullptr, &co, &cb);
        void *blk = nullptr;
        if (hipMalloc(&blk, (size_t)bytes) != hipSuccess) {
            (void)hipGetLastError();
            hps_set_error("hipMalloc of %lld bytes for multi-right-hand-side solve buffers failed", (long long)bytes);
            return HPS_ENOMEM;
        }
        op->allocs.push_back(blk);
        op->total_bytes += bytes;
        Workspace *w = new Workspace();
        workspace_layout(op, (char *)blk, w, &co, &cb);
        if (cb) HPS_HIP(hipMemset((char *)blk + co, 0, (size_t)cb));
        op->mws[k] = w;
    }
    return HPS_OK;
}

// nc right-hand sides (2..4) of an FP64 real operator: one leaf launch up, one level sweep
// and one leaf launch down for all of them, each operator block read once.
static int solve_multi(hps_op *op, int nc, const double *const *body, const double *const *dir,
                       const double *const *jump, double *const *u, hipStream_t st) {
    TRY(multi_workspaces(op, nc - 1));
    const Workspace *ws[MAX_MULTI] = {nullptr, op->mws[0], op->mws[1], op->mws[2]};
    TRY(launch_leaf_multi(op, nc, true, body, nullptr, ws, st));
    TRY(launch_levels_multi(op, nc, ws, dir, jump, st));
    return launch_leaf_multi(op, nc, false, nullptr, u, ws, st);
}

extern "C" int hps_solve(hps_op *op, int nrhs, const double *body, const double *dirichlet,
                         const double *jump, double *u, void *stream, hps_info *info) {
    CHECK_ARG(op != nullptr, "op is NULL");
    CHECK_ARG(nrhs >= 0, "nrhs must be >= 0");
    if (info) *info = hps_info{};
    if (nrhs == 0) return HPS_OK;
    CHECK_ARG(body != nullptr && u != nullptr, "body and u are required");
    TRY(check_device_ptr(body, "body"));
    TRY(check_device_ptr(dirichlet, "dirichlet"));
    TRY(check_device_ptr(jump, "jump"));
    TRY(check_device_ptr(u, "u"));
    hipStream_t st = (hipStream_t)stream;
    const int m = op->ncomp;
    hps_info inf{};
    // FP64 real operators: right-hand sides in groups of up to MAX_MULTI per sweep
    const bool multi = m == 1 && !(op->flags & HPS_FP32_IR) && op->L > 0;
    for (int r = 0; r < nrhs;) {
        int nc = multi ? std::min(MAX_MULTI, nrhs - r) : 1;
        while (nc > 1 && !levels_multi_fit(op, nc)) --nc;
        if (nc > 1) {
            const double *b[MAX_MULTI], *d[MAX_MULTI], *j[MAX_MULTI];
            double *uu[MAX_MULTI];
            for (int c = 0; c < nc; ++c) {
                b[c] = body + (int64_t)(r + c) * op->n_int;
                d[c] = dirichlet ? dirichlet + (int64_t)(r + c) * op->n_bdry : nullptr;
                j[c] = (jump && op->n_iface) ? jump + (int64_t)(r + c) * op->n_iface : nullptr;
                uu[c] = u + (int64_t)(r + c) * op->N;
            }
            TRY(solve_multi(op, nc, b, d, j, uu, st));
            r += nc;
            continue;
        }
        const double *b = body + (int64_t)r * m * op->n_int;
        const double *d = dirichlet ? dirichlet + (int64_t)r * m * op->n_bdry : nullptr;
        const double *j = (jump && op->n_iface) ? jump + (int64_t)r * m * op->n_iface : nullptr;
        double *ur = u + (int64_t)r * m * op->N;
        TRY(solve_one(op, b, d, j, ur, st, &inf));
        ++r;
    }
    if (info) {
        HPS_HIP(hipStreamSynchronize(st));
        *info = inf;
    }
    return HPS_OK;
}

// The leaf launch that opens step phase k of the stage formulation: k = 0 evaluates stage 1
// (L u^n, F_1) and assembles stage 2's right-hand side; k = 1..s-1 closes stage k+1
// (reconstruction, L u, F) and assembles stage k+2's right-hand side, or for the last stage
// the interior update.  qt: device time factors of a separable source (s values).
void hps::step_phase(const ark_ctx *c, int k, double *u, const double *q_stages, const double *q_space,
                     const double *qt, LeafPhase &ph) {
    const hps_op *op = c->op;
    const int s = c->s;
    const int64_t n = op->n_int * op->ncomp;   // one stage vector (both planes when complex)
    ph = LeafPhase{};
    ph.g = GPoly{c->g.kind, c->g.g0, c->g.g1, c->g.g2, c->g.g3};
    ph.q_scale = 1.0;
    if (q_stages) ph.q_src = q_stages + (int64_t)k * n;
    else if (q_space) {
        // the time factors are written to device memory before the step (outside any
        // captured graph), so a replayed step picks up new values
        ph.q_src = q_space;
        ph.q_scale_ptr = qt + k;
    }
    ph.Lu_out = c->Lu + (int64_t)k * n;
    ph.F_out = c->F + (int64_t)k * n;
    if (k == 0) {
        ph.down = LD_EVAL;
        ph.u_eval = u;
    } else {
        ph.down = LD_STAGE;
    }
    ph.un = u;
    ph.Lu_in = c->Lu;
    ph.F_in = c->F;
    if (k + 1 < s) {          // up phase: right-hand side of stage k+2 (index k+1)
        const int i = k + 1;
        ph.up = LU_STAGE;
        ph.nprev = i;
        for (int j = 0; j < i; ++j) {
            ph.ca[j] = c->dt * c->A[i * s + j];
            ph.cf[j] = c->dt * c->Ah[i * s + j];
        }
    } else {                  // up phase: interior u^{n+1}
        ph.up = LU_UPDATE;
        ph.unew = u;
        ph.nprev = s - 1;
        for (int j = 0; j < s; ++j) {
            ph.ca[j] = c->dt * c->b[j];
            ph.cf[j] = c->dt * c->bh[j];
        }
    }
}

// FP32_IR stage solves inside the step: `fixed` > 0 runs that many corrections per stage
// with no host involvement (stage k's pass j writes its folded norms to
// c->ir_stat[(k * IR_MAXIT + j) * 2]); fixed == 0 refines each stage on the host-checked
// loop and redoes a stage that does not converge with the FP64 operators (rec: the
// record of the step).
struct IrStep {
    int fixed = 0;
    hps_info *rec = nullptr;
    bool fp64 = false;   // every stage with the FP64 operators (refinement failed for this operator)
};

static int enqueue_step(ark_ctx *c, double *u, const double *q_stages, const double *q_space,
                        const double *q_time, const double *f_stages, hipStream_t st, IrStep irs = IrStep{}) {
    hps_op *op = c->op;
    const int s = c->s;
    const bool ir = (op->flags & HPS_FP32_IR) != 0 && !irs.fp64;
    (void)q_time;
    if (op->ncomp == 2) {
        // complex operator: u, the boundary data and every stage vector in two planes
        const int64_t nb = op->n_bdry, N = op->N, plane = (int64_t)op->nleaves * 4 * op->q;
        for (int k = 0; k < s; ++k) {
            if (k > 0) TRY(levels(op, false, nullptr, f_stages ? f_stages + (int64_t)k * 2 * nb : nullptr, st));
            LeafPhase ph;
            step_phase(c, k, u, nullptr, nullptr, c->qt_dev, ph);
            TRY(launch_leaf_cx(op, ph, st));
        }
        const double *fend = f_stages ? f_stages + (int64_t)s * 2 * nb : nullptr;
        for (int cc = 0; cc < 2; ++cc)
            TRY(launch_interface_lines(op, u + cc * N, fend ? fend + cc * nb : nullptr, st, nullptr,
                                       op->ir_flux + cc * plane));
        return HPS_OK;
    }
    if (ir && irs.fixed > 0) {
        // a replayed step: keep u^n for a redo, clear the correction norms
        TRY(launch_copy(c->u_save, u, op->N, st));
        TRY(launch_zero(c->ir_stat, (int64_t)s * IR_MAXIT * 2, st));
    }
    for (int k = 0; k < s; ++k) {
        const double *fk = (k > 0 && f_stages) ? f_stages + (int64_t)k * op->n_bdry : nullptr;
        if (k > 0) TRY(levels(op, ir, nullptr, fk, st));
        LeafPhase ph;
        step_phase(c, k, u, q_stages, q_space, c->qt_dev, ph);
        int fold_last = -1;   // a fused last correction: its norms are folded after the launch
        if (ir) {
            if (k > 0) {
                // FP32 stage solve, refined in FP64, then L u_i and F_i from the refined u_i
                LeafPhase w;
                w.down = LD_WRITE_U;
                w.u_out = c->stage_u;
                if (irs.fixed > 0) {
                    // the passes of ir_pass, each residual evaluated in the leaf kernel that
                    // writes u (or adds the previous correction) and whose up phase starts
                    // the next correction's FP32 solve, the last correction added in the
                    // kernel that evaluates L u_i, F_i and opens the next stage: the same
                    // arithmetic in fewer launches
                    w.res_rhs = c->rhs;
                    w.up = LU_BODY;
                    TRY(launch_leaf(op, true, w, st));
                    for (int j = 0; j < irs.fixed; ++j) {
                        if (op->n_iface) {
                            ProfScope ps_(&op->prof, KF_RESIDUAL, st);
                            TRY(launch_flux_jump(op, 1.0, op->ir_r3, st));
                        }
                        TRY(levels(op, true, op->n_iface ? op->ir_r3 : nullptr, nullptr, st));
                        if (j + 1 == irs.fixed) {
                            fold_last = j;
                            break;
                        }
                        LeafPhase dn;
                        dn.down = LD_IR_ADD;
                        dn.u_out = c->stage_u;
                        dn.norm_part = op->ir_part;
                        dn.res_rhs = c->rhs;
                        dn.up = LU_BODY;
                        TRY(launch_leaf(op, true, dn, st));
                        TRY(launch_norm_fold(op->ir_part, (int)op->nleaves, c->ir_stat + ((int64_t)k * IR_MAXIT + j) * 2,
                                             st));
                    }
                    ph.down = LD_IR_ADD;
                    ph.ir_eval = true;
                    ph.u_out = c->stage_u;
                    ph.norm_part = op->ir_part;
                } else {
                    TRY(launch_leaf(op, true, w, st));
                    TRY(ir_finish(op, c->rhs, fk, nullptr, c->stage_u, st, irs.rec));
                    ph.down = LD_EVAL;
                    ph.u_eval = c->stage_u;
                }
            }
            if (k + 1 < s) ph.rhs_copy = c->rhs;
        }
        TRY(launch_leaf(op, ir, ph, st));
        if (fold_last >= 0)
            TRY(launch_norm_fold(op->ir_part, (int)op->nleaves, c->ir_stat + ((int64_t)k * IR_MAXIT + fold_last) * 2, st));
    }
    const double *fend = f_stages ? f_stages + (int64_t)s * op->n_bdry : nullptr;
    TRY(launch_interface_lines(op, u, fend, st));
    return HPS_OK;
}

// One step of the slope formulation with flux-jump penalisation (Sec. 3.1):
//   pen = -[[u^n]]/dt (flux_alpha - flux_beta of u^n), the flux jump every slope gets;
//   k_1: interior L u^n + q_1, boundary fdot_1, interface values from the penalised
//        flux condition (identity equation on the tree: the line solves);
//   l_i = g(u^n + dt sum_{j<=i} a_ij k_j + dt sum_{j<i} ahat_ij l_j), zero on the boundary;
//   (I - gamma dt L) k_i = L u^n + dt sum_{j<i} (a_ij L k_j + ahat_ij L l_j) + q_i with
//        k_i = fdot_i on the boundary and flux jump pen;
//   u^{n+1} = u^n + dt sum_j (b_j k_j + bhat_j l_j) at every node.
static int enqueue_slope_step(ark_ctx *c, double *u, const double *q_stages, const double *q_space,
                              const double *f_dot, hipStream_t st) {
    hps_op *op = c->op;
    const int s = c->s;
    const int64_t n = op->n_int, N = op->N;
    const bool ir = (op->flags & HPS_FP32_IR) != 0;
    const bool nl = c->g.kind != 0;
    const GPoly gp{c->g.kind, c->g.g0, c->g.g1, c->g.g2, c->g.g3};
    const GPoly none{0, 0, 0, 0, 0};
    const double dt = c->dt;
    double *K = c->K, *Ls = c->Ls;
    auto kv = [&](int j) { return K + (int64_t)j * N; };
    auto lv = [&](int j) { return Ls + (int64_t)j * N; };
    auto Lk = [&](int j) { return c->Lk + (int64_t)j * n; };
    auto Ll = [&](int j) { return c->Ll + (int64_t)j * n; };
    auto fd = [&](int i) { return f_dot ? f_dot + (int64_t)i * op->n_bdry : nullptr; };
    auto q_of = [&](int i) -> const double * { return q_stages ? q_stages + (int64_t)i * n : q_space; };
    auto qs_of = [&](int i) -> const double * { return q_space ? c->qt_dev + i : nullptr; };
    const double *pen = op->n_iface ? c->pen : nullptr;
    // L u^n and the penalised jump
    TRY(launch_eval(op, u, c->Lun, true, st));
    if (pen) TRY(launch_flux_jump(op, 1.0 / dt, c->pen, st));
    // k_1: interior values, interior flux parts (edges zero), boundary and interface values
    {
        const double *v[1] = {c->Lun};
        const double cf[1] = {1.0};
        TRY(launch_lincomb(v, cf, 1, q_of(0), qs_of(0), &none, kv(0), n, st));
        TRY(launch_zero(kv(0) + n, N - n, st));
        TRY(launch_eval(op, kv(0), nullptr, true, st));
        TRY(launch_interface_lines(op, kv(0), fd(0), st, pen));
        TRY(launch_eval(op, kv(0), Lk(0), false, st));
    }
    auto make_l = [&](int i) -> int {   // l_i and L l_i
        const double *v[kMaxLinComb];
        double cf[kMaxLinComb];
        int m = 0;
        v[m] = u;
        cf[m++] = 1.0;
        for (int j = 0; j <= i; ++j) {
            v[m] = kv(j);
            cf[m++] = i == 0 ? 0.0 : dt * c->A[i * s + j];
        }
        for (int j = 0; j < i; ++j) {
            v[m] = lv(j);
            cf[m++] = dt * c->Ah[i * s + j];
        }
        TRY(launch_lincomb(v, cf, m, nullptr, nullptr, &gp, lv(i), N, st));
        TRY(launch_scatter_boundary(op, nullptr, lv(i), st));
        TRY(launch_eval(op, lv(i), Ll(i), false, st));
        return HPS_OK;
    };
    if (nl) TRY(make_l(0));
    for (int i = 1; i < s; ++i) {
        const double *v[kMaxLinComb];
        double cf[kMaxLinComb];
        int m = 0;
        v[m] = c->Lun;
        cf[m++] = 1.0;
        for (int j = 0; j < i; ++j) {
            v[m] = Lk(j);
            cf[m++] = dt * c->A[i * s + j];
            if (nl) {
                v[m] = Ll(j);
                cf[m++] = dt * c->Ah[i * s + j];
            }
        }
        TRY(launch_lincomb(v, cf, m, q_of(i), qs_of(i), &none, c->srhs, n, st));
        TRY(solve_one(op, c->srhs, fd(i), pen, kv(i), st, nullptr));
        TRY(launch_eval(op, kv(i), Lk(i), false, st));
        if (nl) TRY(make_l(i));
    }
    const double *v[kMaxLinComb];
    double cf[kMaxLinComb];
    int m = 0;
    v[m] = u;
    cf[m++] = 1.0;
    for (int j = 0; j < s; ++j) {
        v[m] = kv(j);
        cf[m++] = dt * c->b[j];
        if (nl) {
            v[m] = lv(j);
            cf[m++] = dt * c->bh[j];
        }
    }
    (void)ir;
    return launch_lincomb(v, cf, m, nullptr, nullptr, &none, u, N, st);
}

// One step of the two-component Burgers system (Sec. 5.4) in the stage formulation: both
// components share the operator and the tableau; every leaf launch and level sweep runs
// both (each operator block is read once for the two right-hand sides), and the advection
// terms that couple them are evaluated in the leaf kernels.  Component 0 uses the
// operator's solve buffers, component 1 those of its context.
static int enqueue_burgers_step(ark_ctx *cu, ark_ctx *cv, double *u, double *v, const double *fu,
                                const double *fv, hipStream_t st) {
    hps_op *op = cu->op;
    const int s = cu->s;
    const int64_t nb = op->n_bdry;
    const Workspace *ws[2] = {nullptr, cv->ws};
    for (int k = 0; k < s; ++k) {
        if (k > 0) {
            const double *dir[2] = {fu ? fu + (int64_t)k * nb : nullptr, fv ? fv + (int64_t)k * nb : nullptr};
            TRY(launch_levels_sys(op, ws, dir, st));
        }
        LeafPhase p0, p1;
        step_phase(cu, k, u, nullptr, nullptr, cu->qt_dev, p0);
        step_phase(cv, k, v, nullptr, nullptr, cv->qt_dev, p1);
        TRY(launch_leaf_sys(op, p0, p1, ws[0], ws[1], st));
    }
    TRY(launch_interface_lines(op, u, fu ? fu + (int64_t)s * nb : nullptr, st));
    TRY(launch_interface_lines(op, v, fv ? fv + (int64_t)s * nb : nullptr, st, nullptr, cv->ws->flux));
    return HPS_OK;
}

// Enqueue one step.  A step without host synchronisation (FP64; FP32_IR with a fixed
// number of corrections) is captured once into a HIP graph (kept in c) and replayed while
// `key` (the formulation and the array arguments) repeats.  Host-checked refinement and
// profiled steps run eagerly.
template <typename Enqueue>
static int run_captured(ark_ctx *c, const std::vector<uintptr_t> &key, Enqueue enqueue, hipStream_t st,
                        bool capturable = true) {
    hps_op *op = c->op;
    const char *env = getenv("HPS_GRAPHS");
    const bool graphs = capturable && !(env && env[0] == '0') && !op->prof.on;
    if (!graphs) return enqueue(st);
    if (!c->gexec || key != c->gkey) {
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->gexec = nullptr;
        c->graph = nullptr;
        c->gkey.clear();
        // capture on a private stream (the legacy default stream cannot be captured); the
        // instantiated graph is then launched on the caller's stream
        if (!c->cap_stream) HPS_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HPS_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        int rc = enqueue(c->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        HPS_HIP(e);
        c->graph = g;
        HPS_HIP(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
        c->gkey = key;
    }
    HPS_HIP(hipGraphLaunch(c->gexec, st));
    return HPS_OK;
}

// The stage formulation on an FP32_IR operator.  The first step (and a profiled one)
// refines every stage on the host-checked loop and records the most corrections a stage
// needed; later steps replay a captured graph with that many corrections per stage, then
// wait for the stream and read every stage's last correction norm.  A stage that missed
// the tolerance makes the step be redone from the saved u^n on the host-checked loop,
// with FP64 re-solves where needed (HPS_IR_STRICT: HPS_ENOTCONVERGED), and the next
// captured steps run one correction more.  Once a stage had to be re-solved in FP64, the
// refinement is taken to fail for this operator: later steps use the FP64 operators only
// (replayed like an FP64 step).
static int run_step_ir(ark_ctx *c, double *u, const double *q_stages, const double *q_space, const double *q_time,
                       const double *f, hipStream_t st) {
    hps_op *op = c->op;
    const int s = c->s;
    const char *env = getenv("HPS_GRAPHS");
    const bool graphs = !(env && env[0] == '0') && !op->prof.on;
    if (c->ir_passes < 0) {
        IrStep irs;
        irs.fp64 = true;
        const std::vector<uintptr_t> key = {(uintptr_t)4, (uintptr_t)u, (uintptr_t)q_stages, (uintptr_t)q_space,
                                            (uintptr_t)f};
        TRY(run_captured(c, key, [&](hipStream_t s2) { return enqueue_step(c, u, q_stages, q_space, q_time, f, s2, irs); },
                         st));
        c->last = hps_info{0, 0.0, s - 1};
        return HPS_OK;
    }
    auto eager = [&]() -> int {
        hps_info rec{};
        IrStep irs;
        irs.rec = &rec;
        const int rc = enqueue_step(c, u, q_stages, q_space, q_time, f, st, irs);
        c->last = rec;
        if (rc) return rc;
        if (rec.fp64_fallbacks > 0) c->ir_passes = -1;
        else c->ir_passes = std::min(IR_MAXIT, std::max(c->ir_passes, rec.ir_iterations));
        return HPS_OK;
    };
    if (!graphs || c->ir_passes == 0) return eager();
    const int K = c->ir_passes;
    const std::vector<uintptr_t> key = {(uintptr_t)3, (uintptr_t)u, (uintptr_t)q_stages, (uintptr_t)q_space,
                                        (uintptr_t)f, (uintptr_t)K};
    IrStep irs;
    irs.fixed = K;
    TRY(run_captured(c, key, [&](hipStream_t s2) { return enqueue_step(c, u, q_stages, q_space, q_time, f, s2, irs); },
                     st));
    std::vector<unsigned long long> nb((size_t)s * IR_MAXIT * 2);
    HPS_HIP(hipMemcpyAsync(nb.data(), c->ir_stat, nb.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HPS_HIP(hipStreamSynchronize(st));
    return ir_step_finish(c, u, q_stages, q_space, q_time, f, st, nb.data());
}

// After a step with c->ir_passes fixed corrections per stage (stats: the step's correction
// norms, copied from c->ir_stat once the step has completed): record the step, and if a
// stage missed the tolerance redo the step from the saved u^n on the host-checked loop
// (HPS_IR_STRICT: HPS_ENOTCONVERGED); later steps then run one correction more.
int hps::ir_step_finish(ark_ctx *c, double *u, const double *q_stages, const double *q_space, const double *q_time,
                        const double *f, hipStream_t st, const unsigned long long *stats) {
    hps_op *op = c->op;
    const int s = c->s, K = c->ir_passes;
    hps_info rec{};
    rec.ir_iterations = K;
    bool all = true;
    for (int k = 1; k < s; ++k) {
        double rel = 0.0;
        all = ir_converged(&stats[((size_t)k * IR_MAXIT + K - 1) * 2], &rel) && all;
        rec.last_correction = std::max(rec.last_correction, rel);
    }
    c->last = rec;
    if (all) return HPS_OK;
    if (op->flags & HPS_IR_STRICT) {
        hps_set_error("iterative refinement did not converge within %d corrections: last correction %.3e", K,
                      rec.last_correction);
        return HPS_ENOTCONVERGED;
    }
    // redo the step from u^n with host-checked refinement
    TRY(launch_copy(u, c->u_save, op->N, st));
    hps_info redo{};
    IrStep irs;
    irs.rec = &redo;
    TRY(enqueue_step(c, u, q_stages, q_space, q_time, f, st, irs));
    c->last = redo;
    if (redo.fp64_fallbacks > 0) c->ir_passes = -1;
    else c->ir_passes = std::min(IR_MAXIT, std::max(K + 1, redo.ir_iterations));
    return HPS_OK;
}

static int run_step(ark_ctx *c, int mode, double *u, const double *q_stages, const double *q_space,
                    const double *q_time, const double *f, hipStream_t st) {
    if (q_space) TRY(launch_set_values(c->qt_dev, q_time, c->s, st));
    const bool ir = (c->op->flags & HPS_FP32_IR) != 0;
    if (ir && mode == 0) return run_step_ir(c, u, q_stages, q_space, q_time, f, st);
    auto enqueue = [&](hipStream_t s2) {
        return mode == 0 ? enqueue_step(c, u, q_stages, q_space, q_time, f, s2)
                         : enqueue_slope_step(c, u, q_stages, q_space, f, s2);
    };
    const std::vector<uintptr_t> key = {(uintptr_t)mode, (uintptr_t)u, (uintptr_t)q_stages, (uintptr_t)q_space,
                                        (uintptr_t)f};
    // the slope formulation's FP32_IR solves refine on the host-checked loop
    return run_captured(c, key, enqueue, st, !ir);
}

extern "C" int ark_info(const ark_ctx *c, hps_info *info) {
    CHECK_ARG(c != nullptr && info != nullptr, "ctx and info are required");
    *info = c->last;
    return HPS_OK;
}

static int check_step_args(ark_ctx *c, double t, double *u, const double *q_stages, const double *q_space,
                           const double *q_time, const double *f) {
    CHECK_ARG(c != nullptr && u != nullptr, "ctx and u are required");
    CHECK_ARG(std::isfinite(t), "t must be finite");
    CHECK_ARG(!(q_stages && q_space), "give q_stages or q_space/q_time, not both");
    CHECK_ARG(!q_space || q_time, "q_space needs q_time (host array of s values)");
    TRY(check_device_ptr(u, "u"));
    TRY(check_device_ptr(q_stages, "q_stages"));
    TRY(check_device_ptr(q_space, "q_space"));
    TRY(check_device_ptr(f, "boundary data"));
    return HPS_OK;
}

extern "C" int ark_step(ark_ctx *c, double t, double *u, const double *q_stages, const double *q_space,
                        const double *q_time, const double *f_stages, void *stream) {
    TRY(check_step_args(c, t, u, q_stages, q_space, q_time, f_stages));
    CHECK_ARG(c->op->ncomp == 1 || (!q_stages && !q_space), "steps of a complex operator take no source");
    return run_step(c, 0, u, q_stages, q_space, q_time, f_stages, (hipStream_t)stream);
}

extern "C" int ark_step_slope(ark_ctx *c, double t, double *u, const double *q_stages, const double *q_space,
                              const double *q_time, const double *fdot_stages, void *stream) {
    TRY(check_step_args(c, t, u, q_stages, q_space, q_time, fdot_stages));
    CHECK_ARG(c->s <= 8, "the slope step takes at most 8 stages");
    CHECK_ARG(c->op->ncomp == 1, "the slope step takes a real operator");
    TRY(ark_slope_workspace(c));
    return run_step(c, 1, u, q_stages, q_space, q_time, fdot_stages, (hipStream_t)stream);
}

extern "C" int ark_step_burgers(ark_ctx *cu, ark_ctx *cv, double t, double *u, double *v,
                                const double *fu_stages, const double *fv_stages, void *stream) {
    CHECK_ARG(cu != nullptr && cv != nullptr && u != nullptr && v != nullptr, "cu, cv, u and v are required");
    CHECK_ARG(cu != cv, "the two components need a context each");
    CHECK_ARG(u != v, "u and v must be different arrays");
    CHECK_ARG(cu->op == cv->op, "both contexts must be created on the same operator");
    CHECK_ARG(!(cu->op->flags & HPS_FP32_IR) && cu->op->ncomp == 1,
              "two-component steps need a real operator built with HPS_FP64");
    CHECK_ARG(cu->s == cv->s && cu->dt == cv->dt && cu->A == cv->A && cu->b == cv->b && cu->c == cv->c &&
                  cu->Ah == cv->Ah && cu->bh == cv->bh,
              "both contexts must have the same tableau and dt");
    CHECK_ARG(cu->g.kind == 0 && cv->g.kind == 0, "the advection terms replace g: create both contexts with g = NULL");
    CHECK_ARG(std::isfinite(t), "t must be finite");
    TRY(check_device_ptr(u, "u"));
    TRY(check_device_ptr(v, "v"));
    TRY(check_device_ptr(fu_stages, "fu_stages"));
    TRY(check_device_ptr(fv_stages, "fv_stages"));
    TRY(ctx_workspace(cv));
    const std::vector<uintptr_t> key = {(uintptr_t)2,         (uintptr_t)u,         (uintptr_t)v,
                                        (uintptr_t)fu_stages, (uintptr_t)fv_stages, (uintptr_t)cv,
                                        (uintptr_t)cv->uid};
    return run_captured(cu, key, [&](hipStream_t s2) { return enqueue_burgers_step(cu, cv, u, v, fu_stages, fv_stages, s2); },
                        (hipStream_t)stream);
}
