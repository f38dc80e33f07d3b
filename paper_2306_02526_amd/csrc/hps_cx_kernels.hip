// Per-leaf kernels for complex operators (the regularised NLS of Sec. 5.5).
//
// A complex operator is stored as its real embedding: every leaf's A_ii^{-1} is
// 2 q^2 x 2 q^2 acting on [Re | Im] of the interior values, S_leaf maps the leaf boundary
// [Re edges | Im edges] to the interior, and the merge levels carry both parts in their
// (doubled) index sets, so the level kernels of the real solve run unchanged.  Vectors of
// the caller are two planes of the real layout (real part, then imaginary part).
//
// One workgroup per leaf runs the down phase of the stage that ends here (reconstruct
// u_i = S_leaf u_b + w, then L u_i and F_i = g(u_i) with complex coefficients) and the up
// phase of the next one (rhs = u^n + dt sum_j (a_ij L u_j + ahat_ij F_j), w = A_ii^{-1} rhs,
// fluxes h of both parts), or the interior update, exactly as the real kernels do for one
// part; the plain solve phases (body -> w, h; reconstruct and write u) are the same.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hps_device.h"

namespace hps {

namespace {

constexpr int CPF = 2;    // operator loads issued ahead of each stream
constexpr int CUNR = 8;   // operator loads in flight in the streaming loop

struct LeafCxArgs {
    LeafGeo geo;
    int64_t N;                      // length of one plane of a full vector
    const int *leaf_ij;
    const double *D, *D2, *coef;    // coef: 5 real planes, then 5 imaginary planes
    int xs_cap, part_cap;
    PanelView sl, ainv;
    const double *ub, *w_in;        // [leaf][8q], [leaf][2 q^2]
    const double *u_eval;           // LD_EVAL: two planes of N
    double *u_out;                  // LD_WRITE_U: two planes of N
    double *Lu_out, *F_out;         // two planes of n_int each
    GPoly g;                        // kind 2: g(u) = (g0 + i g1) u + (g2 + i g3) |u|^2 u
    const double *body;             // LU_BODY: two planes of n_int
    const double *un;               // two planes of N
    const double *Lu_in, *F_in;     // stage j, part c at (2 j + c) n_int
    int nprev;
    double ca[8], cf[8];
    double *w_out, *h_out;          // [leaf][2 q^2], [leaf][8q]
    double *unew;                   // LU_UPDATE: two planes of N
    double *fpart;                  // LU_UPDATE: two planes of [leaf (canonical)][4q]
};

// Sum the column-group partials of `rows` rows (LDS, [g][rows]), then fin(row, y), in a
// fixed order.
template <typename Fin>
__device__ __forceinline__ void sum_rows(const double *part, int rows, int G, double *red, Fin fin) {
    for (int r0 = 0; r0 < rows; r0 += NT) {
        const int nr = min(NT, rows - r0);
        const int nsl = min(G, NT / nr);
        const int t = threadIdx.x;
        const int row = t % nr, sl = t / nr;
        if (sl < nsl) {
            double y = 0.0;
            for (int gg = sl; gg < G; gg += nsl) y += part[gg * rows + r0 + row];
            red[sl * nr + row] = y;
        }
        __syncthreads();
        if (t < nr) {
            double y = 0.0;
            for (int s2 = 0; s2 < nsl; ++s2) y += red[s2 * nr + t];
            fin(r0 + t, y);
        }
        __syncthreads();
    }
}

template <int DN, int UPM>
__device__ __forceinline__ void leaf_cx_body(const LeafCxArgs &a, int leaf, unsigned char *smem, double *red) {
    constexpr int VW = 2;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q, pp = p * p;
    const int nil = 2 * q2, nbl = 2 * nb;
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int64_t n_int = a.geo.n_int, N = a.N;
    Carve cv{smem};
    double *xs = cv.take<double>(a.xs_cap);
    double *part = cv.take<double>(a.part_cap);
    double *tile = cv.take<double>(2 * (size_t)pp);   // [part][p*p]
    const int ld = dmat_ld(p);
    double *D = cv.take<double>((size_t)p * ld);
    double *D2 = cv.take<double>((size_t)p * ld);
    double *luv = cv.take<double>(2 * (size_t)q2);    // [part][q2]
    double *fv = cv.take<double>(2 * (size_t)q2);
    constexpr bool stream_down = DN == LD_WRITE_U || DN == LD_STAGE;
    constexpr bool stream_up = UPM == LU_BODY || UPM == LU_STAGE;
    constexpr bool need_L = DN == LD_STAGE || DN == LD_EVAL;
    PanelStream<double, CPF, CUNR> ps;
    if constexpr (stream_down)
        ps.start(reinterpret_cast<const double *>(a.sl.data) + (int64_t)leaf * a.sl.node_elems, a.sl.rp, a.sl.G,
                 a.sl.S, a.sl.node_elems == 0);
    else if constexpr (stream_up)
        ps.start(reinterpret_cast<const double *>(a.ainv.data) + (int64_t)leaf * a.ainv.node_elems, a.ainv.rp,
                 a.ainv.G, a.ainv.S, a.ainv.node_elems == 0);
    load_dmat_ld(a.D, D, p);
    if (need_L) load_dmat_ld(a.D2, D2, p);

    // ---------------- down phase ----------------
    if constexpr (DN != LD_NONE) {
        for (int k = threadIdx.x; k < 2 * pp; k += NT) tile[k] = 0.0;
        if constexpr (stream_down) {
            const double *ubl = a.ub + (int64_t)leaf * nbl;
            for (int k = threadIdx.x; k < nil; k += NT) fv[k] = a.w_in[(int64_t)leaf * nil + k];
            const int SG = a.sl.S * a.sl.G;
            for (int k = threadIdx.x; k < SG; k += NT) xs[k] = k < nbl ? ubl[k] : 0.0;
            __syncthreads();
            for (int k = threadIdx.x; k < nbl; k += NT) {
                const int c = k / nb, kk = k % nb;
                tile[c * pp + edge_tile_pos(p, q, kk / q, kk % q)] = ubl[k];
            }
            ps.finish(xs, part);
            if constexpr (stream_up)
                ps.start(reinterpret_cast<const double *>(a.ainv.data) + (int64_t)leaf * a.ainv.node_elems, a.ainv.rp,
                         a.ainv.G, a.ainv.S, a.ainv.node_elems == 0);
            __syncthreads();
            // interior of both parts: u = S_leaf u_b + w
            sum_rows(part, a.sl.rp * VW, a.sl.G, red, [&](int row, double y) {
                if (row < nil) {
                    const int c = row / q2, r = row % q2;
                    tile[c * pp + (r / q + 1) * p + (r % q) + 1] = y + fv[row];
                }
            });
        } else {
            __syncthreads();
            for (int c = 0; c < 2; ++c) {
                const double *ue = a.u_eval + c * N;
                for (int k = threadIdx.x; k < q2; k += NT) tile[c * pp + (k / q + 1) * p + (k % q) + 1] = ue[base + k];
                for (int k = threadIdx.x; k < nb; k += NT)
                    tile[c * pp + edge_tile_pos(p, q, k / q, k % q)] = ue[edge_index(a.geo, li, lj, k / q, k % q)];
            }
            __syncthreads();
        }
        if constexpr (need_L) {
            for (int k = threadIdx.x; k < q2; k += NT) {
                const int aa = k % q + 1, bb = k / q + 1;
                double d[2][5];   // u_xx, u_yy, u_x, u_y, u of each part
                for (int c = 0; c < 2; ++c) {
                    const double *tc = tile + c * pp;
                    double ux = 0, uxx = 0, uy = 0, uyy = 0;
                    for (int m = 0; m < p; ++m) {
                        const double xr = tc[bb * p + m];
                        const double yc = tc[m * p + aa];
                        ux = fma(D[aa * ld + m], xr, ux);
                        uxx = fma(D2[aa * ld + m], xr, uxx);
                        uy = fma(D[bb * ld + m], yc, uy);
                        uyy = fma(D2[bb * ld + m], yc, uyy);
                    }
                    d[c][0] = uxx; d[c][1] = uyy; d[c][2] = ux; d[c][3] = uy; d[c][4] = tc[bb * p + aa];
                }
                // L u = sum_k (cr_k + i ci_k)(d_re,k + i d_im,k)  (eq. 3 with complex coefficients)
                double Lr = 0.0, Li = 0.0;
                for (int t = 0; t < 5; ++t) {
                    const double cr = a.coef[t * n_int + base + k], ci = a.coef[(5 + t) * n_int + base + k];
                    Lr += cr * d[0][t] - ci * d[1][t];
                    Li += cr * d[1][t] + ci * d[0][t];
                }
                const double ur = d[0][4], ui = d[1][4];
                double Fr = 0.0, Fi = 0.0;
                if (a.g.kind == 2) {
                    const double rho = ur * ur + ui * ui;
                    Fr = a.g.g0 * ur - a.g.g1 * ui + rho * (a.g.g2 * ur - a.g.g3 * ui);
                    Fi = a.g.g0 * ui + a.g.g1 * ur + rho * (a.g.g2 * ui + a.g.g3 * ur);
                }
                luv[k] = Lr;
                luv[q2 + k] = Li;
                fv[k] = Fr;
                fv[q2 + k] = Fi;
                a.Lu_out[base + k] = Lr;
                a.Lu_out[n_int + base + k] = Li;
                a.F_out[base + k] = Fr;
                a.F_out[n_int + base + k] = Fi;
            }
        } else if constexpr (DN == LD_WRITE_U) {
            const double *ubl = a.ub + (int64_t)leaf * nbl;
            for (int c = 0; c < 2; ++c) {
                for (int k = threadIdx.x; k < q2 + nb; k += NT) {
                    int64_t gi;
                    double v;
                    if (k < q2) {
                        gi = base + k;
                        v = tile[c * pp + (k / q + 1) * p + (k % q) + 1];
                    } else {
                        const int e = (k - q2) / q, m = (k - q2) % q;
                        // each edge node is written by exactly one leaf
                        const bool own = (e == 0 || e == 2) || (e == 1 && li == a.geo.n1 - 1) ||
                                         (e == 3 && lj == a.geo.n2 - 1);
                        if (!own) continue;
                        gi = edge_index(a.geo, li, lj, e, m);
                        v = ubl[c * nb + k - q2];
                    }
                    a.u_out[c * N + gi] = v;
                }
            }
        }
        __syncthreads();
    }

    // ---------------- up phase ----------------
    if constexpr (UPM == LU_NONE) return;
    if constexpr (UPM == LU_UPDATE) {
        const int last = a.nprev;
        for (int c = 0; c < 2; ++c) {
            double *vals = tile + c * pp;   // interior values of u^{n+1}, row-major q x q
            for (int k = threadIdx.x; k < q2; k += NT) {
                double v = a.un[c * N + base + k];
                for (int j = 0; j < last; ++j) {
                    v += a.ca[j] * a.Lu_in[(2 * j + c) * n_int + base + k];
                    v += a.cf[j] * a.F_in[(2 * j + c) * n_int + base + k];
                }
                v += a.ca[last] * luv[c * q2 + k] + a.cf[last] * fv[c * q2 + k];
                a.unew[c * N + base + k] = v;
                vals[k] = v;
            }
        }
        __syncthreads();
        const int64_t plane = (int64_t)a.geo.n1 * a.geo.n2 * nb;
        for (int c = 0; c < 2; ++c) {
            const double *vals = tile + c * pp;
            for (int k = threadIdx.x; k < nb; k += NT) {
                const int e = k / q, m = k % q;
                const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * ld);
                double f = 0.0;
                if (e < 2) {
                    for (int cc = 1; cc <= q; ++cc) f = fma(dr[cc], vals[m * q + cc - 1], f);
                } else {
                    for (int cc = 1; cc <= q; ++cc) f = fma(dr[cc], vals[(cc - 1) * q + m], f);
                }
                a.fpart[c * plane + ((int64_t)lj * a.geo.n1 + li) * nb + k] = f;
            }
        }
        return;
    }
    const int SG = a.ainv.S * a.ainv.G;
    for (int k = threadIdx.x; k < SG; k += NT) {
        double r = 0.0;
        if (k < nil) {
            const int c = k / q2, kk = k % q2;
            if (UPM == LU_BODY) {
                r = a.body[c * n_int + base + kk];
            } else {
                r = a.un[c * N + base + kk];
                const int last = a.nprev - 1;   // newest stage, held in LDS
                for (int j = 0; j < last; ++j) {
                    r += a.ca[j] * a.Lu_in[(2 * j + c) * n_int + base + kk];
                    r += a.cf[j] * a.F_in[(2 * j + c) * n_int + base + kk];
                }
                r += a.ca[last] * luv[k] + a.cf[last] * fv[k];
            }
        }
        xs[k] = r;
    }
    __syncthreads();
    ps.finish(xs, part);
    __syncthreads();
    double *wv = luv;   // w = A_ii^{-1} rhs of both parts; luv is free again
    sum_rows(part, a.ainv.rp * VW, a.ainv.G, red, [&](int row, double y) {
        if (row < nil) {
            wv[row] = y;
            a.w_out[(int64_t)leaf * nil + row] = y;
        }
    });
    for (int k = threadIdx.x; k < nbl; k += NT) {
        const int c = k / nb, kk = k % nb;
        const int e = kk / q, m = kk % q;
        const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * ld);
        const double *w = wv + c * q2;
        double h = 0.0;
        if (e < 2) {
            for (int cc = 1; cc <= q; ++cc) h = fma(dr[cc], w[m * q + cc - 1], h);
        } else {
            for (int cc = 1; cc <= q; ++cc) h = fma(dr[cc], w[(cc - 1) * q + m], h);
        }
        a.h_out[(int64_t)leaf * nbl + k] = h;
    }
}

template <int DN, int UPM>
__global__ __launch_bounds__(NT) void k_leaf_cx(LeafCxArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT];
    leaf_cx_body<DN, UPM>(a, blockIdx.x, smem, red);
}

}  // namespace

int launch_leaf_cx(const hps_op *op, const LeafPhase &ph, hipStream_t st) {
    const int fam = ph.down == LD_EVAL ? KF_LEAFC_EVAL_UP64
                    : ph.down == LD_STAGE ? (ph.up == LU_UPDATE ? KF_LEAFC_DOWN_UPDATE64 : KF_LEAFC_DOWN_UP64)
                                          : KF_LEAFC_SOLVE64;
    ProfScope ps_(&op->prof, fam, st);
    LeafCxArgs a{};
    a.geo = geo_of(op);
    a.N = op->N;
    a.leaf_ij = op->leaf_ij;
    a.D = op->D;
    a.D2 = op->D2;
    a.coef = op->coef;
    a.sl = view(op->sleaf64);
    a.ainv = view(op->ainv64);
    a.xs_cap = std::max(op->sleaf64.S * op->sleaf64.G, op->ainv64.S * op->ainv64.G);
    a.part_cap = std::max(op->sleaf64.G * op->sleaf64.rp, op->ainv64.G * op->ainv64.rp) * 2;
    a.ub = op->ub_leaf;
    a.w_in = op->w_leaf;
    a.u_eval = ph.u_eval;
    a.u_out = ph.u_out;
    a.Lu_out = ph.Lu_out;
    a.F_out = ph.F_out;
    a.g = ph.g;
    a.body = ph.body;
    a.un = ph.un;
    a.Lu_in = ph.Lu_in;
    a.F_in = ph.F_in;
    a.nprev = ph.nprev;
    for (int j = 0; j < 8; ++j) {
        a.ca[j] = ph.ca[j];
        a.cf[j] = ph.cf[j];
    }
    a.w_out = op->w_leaf;
    a.h_out = op->h_leaf;
    a.unew = ph.unew;
    a.fpart = op->ir_flux;
    const size_t pp = (size_t)op->p * op->p * 8, pd = (size_t)op->p * dmat_ld(op->p) * 8, q2b = (size_t)op->q2 * 8;
    const size_t lds = carve_bytes({(size_t)a.xs_cap * 8, (size_t)a.part_cap * 8, 2 * pp, pd, pd, 2 * q2b, 2 * q2b});
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(op->nleaves), dim3(NT), lds, st, a); };
#define HPS_LEAF_CX_CASE(DNV, UPV)                      \
    if (ph.down == DNV && ph.up == UPV) {               \
        go(k_leaf_cx<DNV, UPV>);                        \
        HPS_LAUNCHED();                                 \
        return HPS_OK;                                  \
    }
    HPS_LEAF_CX_CASE(LD_EVAL, LU_STAGE)
    HPS_LEAF_CX_CASE(LD_STAGE, LU_STAGE)
    HPS_LEAF_CX_CASE(LD_STAGE, LU_UPDATE)
    HPS_LEAF_CX_CASE(LD_NONE, LU_BODY)
    HPS_LEAF_CX_CASE(LD_WRITE_U, LU_NONE)
#undef HPS_LEAF_CX_CASE
    hps_set_error("internal: unsupported complex leaf phase combination (%d, %d)", ph.down, ph.up);
    return HPS_EINVAL;
}

}  // namespace hps
