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

// FP32 operators inside FP64 iterative refinement: u = HPS32(rhs) has been computed;
// repeat { r = FP64 residual of the global system (interior rows and interface flux
// jumps); u += HPS32(r) } until max|delta| <= tol max|u|.
static int ir_refine(hps_op *op, const double *rhs, const double *jump, double *u, hipStream_t st,
                     hps_info *info) {
    const double tol = 1e-11;
    const int maxit = 10;
    int it = 0;
    double rel = 0.0;
    for (it = 1; it <= maxit; ++it) {
        TRY(launch_residual(op, u, rhs, jump, op->ir_r, op->ir_r3, st));
        HPS_HIP(hipMemsetAsync(op->ir_norms, 0, 2 * sizeof(double), st));
        LeafPhase up;
        up.up = LU_BODY;
        up.body = op->ir_r;
        TRY(launch_leaf(op, true, up, st));
        TRY(levels(op, true, op->n_iface ? op->ir_r3 : nullptr, nullptr, st));
        LeafPhase dn;
        dn.down = LD_IR_ADD;
        dn.u_out = u;
        TRY(launch_leaf(op, true, dn, st));
        unsigned long long nb[2];
        HPS_HIP(hipMemcpyAsync(nb, op->ir_norms, sizeof(nb), hipMemcpyDeviceToHost, st));
        HPS_HIP(hipStreamSynchronize(st));
        const double dmax = ordered_bits_to_double(nb[0]), umax = ordered_bits_to_double(nb[1]);
        rel = umax > 0 ? dmax / umax : dmax;
        if (dmax <= tol * umax) break;
    }
    if (info) {
        info->ir_iterations = std::min(it, maxit);
        info->last_correction = rel;
    }
    if (it > maxit) {
        hps_set_error("iterative refinement did not converge: last correction %.3e", rel);
        return HPS_ENOTCONVERGED;
    }
    return HPS_OK;
}

extern "C" int hps_solve(hps_op *op, int nrhs, const double *body, const double *dirichlet,
                         const double *jump, double *u, void *stream, hps_info *info) {
    CHECK_ARG(op != nullptr, "op is NULL");
    CHECK_ARG(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return HPS_OK;
    CHECK_ARG(body != nullptr && u != nullptr, "body and u are required");
    TRY(check_device_ptr(body, "body"));
    TRY(check_device_ptr(dirichlet, "dirichlet"));
    TRY(check_device_ptr(jump, "jump"));
    TRY(check_device_ptr(u, "u"));
    hipStream_t st = (hipStream_t)stream;
    const bool ir = (op->flags & HPS_FP32_IR) != 0;
    int worst_it = 0;
    double worst_rel = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        const double *b = body + (int64_t)r * op->n_int;
        const double *d = dirichlet ? dirichlet + (int64_t)r * op->n_bdry : nullptr;
        const double *j = (jump && op->n_iface) ? jump + (int64_t)r * op->n_iface : nullptr;
        double *ur = u + (int64_t)r * op->N;
        LeafPhase up;
        up.up = LU_BODY;
        up.body = b;
        TRY(launch_leaf(op, ir, up, st));
        TRY(levels(op, ir, j, d, st));
        LeafPhase dn;
        dn.down = LD_WRITE_U;
        dn.u_out = ur;
        TRY(launch_leaf(op, ir, dn, st));
        if (ir) {
            hps_info inf{};
            TRY(ir_refine(op, b, j, ur, st, &inf));
            worst_it = std::max(worst_it, inf.ir_iterations);
            worst_rel = std::max(worst_rel, inf.last_correction);
        }
    }
    if (info) {
        HPS_HIP(hipStreamSynchronize(st));
        info->ir_iterations = worst_it;
        info->last_correction = worst_rel;
    }
    return HPS_OK;
}

static int enqueue_step(ark_ctx *c, double *u, const double *q_stages, const double *q_space,
                        const double *q_time, const double *f_stages, hipStream_t st) {
    hps_op *op = c->op;
    const int s = c->s;
    const int64_t n = op->n_int;
    const bool ir = (op->flags & HPS_FP32_IR) != 0;
    const GPoly gp{c->g.kind, c->g.g0, c->g.g1, c->g.g2, c->g.g3};
    // source of stage i and the coefficients that assemble stage i's right-hand side
    auto set_q = [&](LeafPhase &ph, int i) {
        ph.g = gp;
        ph.q_scale = 1.0;
        ph.q_src = nullptr;
        if (q_stages) ph.q_src = q_stages + (int64_t)i * n;
        else if (q_space) {
            // the time factors are written to c->qt_dev before the step (outside any
            // captured graph), so a replayed step picks up new values
            ph.q_src = q_space;
            ph.q_scale_ptr = c->qt_dev + i;
        }
    };
    auto set_rhs = [&](LeafPhase &ph, int i) {   // up phase: right-hand side of stage i
        ph.up = LU_STAGE;
        ph.un = u;
        ph.Lu_in = c->Lu;
        ph.F_in = c->F;
        ph.nprev = i;
        for (int j = 0; j < i; ++j) {
            ph.ca[j] = c->dt * c->A[i * s + j];
            ph.cf[j] = c->dt * c->Ah[i * s + j];
        }
    };
    auto set_update = [&](LeafPhase &ph) {       // up phase: interior u^{n+1}
        ph.up = LU_UPDATE;
        ph.un = u;
        ph.unew = u;
        ph.Lu_in = c->Lu;
        ph.F_in = c->F;
        ph.nprev = s - 1;
        for (int j = 0; j < s; ++j) {
            ph.ca[j] = c->dt * c->b[j];
            ph.cf[j] = c->dt * c->bh[j];
        }
    };
    // stage 1 is explicit: L u^n and F_1, fused with the right-hand side of stage 2
    {
        LeafPhase ph;
        ph.down = LD_EVAL;
        ph.u_eval = u;
        ph.Lu_out = c->Lu;
        ph.F_out = c->F;
        set_q(ph, 0);
        set_rhs(ph, 1);
        if (ir) ph.rhs_copy = c->rhs;
        TRY(launch_leaf(op, ir, ph, st));
    }
    for (int i = 1; i < s; ++i) {
        const double *fi = f_stages ? f_stages + (int64_t)i * op->n_bdry : nullptr;
        TRY(levels(op, ir, nullptr, fi, st));
        LeafPhase ph;
        set_q(ph, i);
        ph.Lu_out = c->Lu + (int64_t)i * n;
        ph.F_out = c->F + (int64_t)i * n;
        if (!ir) {
            ph.down = LD_STAGE;
        } else {
            // FP32 stage solve, refined in FP64, then L u_i and F_i from the refined u_i
            LeafPhase w;
            w.down = LD_WRITE_U;
            w.u_out = c->stage_u;
            TRY(launch_leaf(op, true, w, st));
            TRY(ir_refine(op, c->rhs, nullptr, c->stage_u, st, nullptr));
            ph.down = LD_EVAL;
            ph.u_eval = c->stage_u;
        }
        if (i + 1 < s) {
            set_rhs(ph, i + 1);
            if (ir) ph.rhs_copy = c->rhs;
        } else {
            set_update(ph);
        }
        TRY(launch_leaf(op, ir, ph, st));
    }
    const double *fend = f_stages ? f_stages + (int64_t)s * op->n_bdry : nullptr;
    TRY(launch_interface_lines(op, u, fend, st));
    return HPS_OK;
}

extern "C" int ark_step(ark_ctx *c, double t, double *u, const double *q_stages, const double *q_space,
                        const double *q_time, const double *f_stages, void *stream) {
    CHECK_ARG(c != nullptr && u != nullptr, "ctx and u are required");
    CHECK_ARG(std::isfinite(t), "t must be finite");
    CHECK_ARG(!(q_stages && q_space), "give q_stages or q_space/q_time, not both");
    CHECK_ARG(!q_space || q_time, "q_space needs q_time (host array of s values)");
    TRY(check_device_ptr(u, "u"));
    TRY(check_device_ptr(q_stages, "q_stages"));
    TRY(check_device_ptr(q_space, "q_space"));
    TRY(check_device_ptr(f_stages, "f_stages"));
    hipStream_t st = (hipStream_t)stream;
    hps_op *op = c->op;
    if (q_space) TRY(launch_set_values(c->qt_dev, q_time, c->s, st));
    // The FP64 step has no host synchronisation, so it is captured once into a HIP graph
    // and replayed while its array arguments repeat.  The
    // refinement loop of FP32_IR waits on the host and runs eagerly; so does a profiled step.
    const char *env = getenv("HPS_GRAPHS");
    const bool graphs = !(env && env[0] == '0') && !(op->flags & HPS_FP32_IR) && !op->prof.on;
    if (!graphs) return enqueue_step(c, u, q_stages, q_space, q_time, f_stages, st);
    const std::vector<uintptr_t> key = {(uintptr_t)u, (uintptr_t)q_stages, (uintptr_t)q_space, (uintptr_t)f_stages};
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
        int rc = enqueue_step(c, u, q_stages, q_space, q_time, f_stages, c->cap_stream);
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
