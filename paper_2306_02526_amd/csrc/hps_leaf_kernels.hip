// Per-leaf kernels of the stage solve, fused across stage boundaries.
//
// One workgroup per leaf runs a "down" phase and then an "up" phase:
//   down: u_i = S_leaf u_b + w (Algorithm 1 with the particular part, Sec. 2.1) followed by
//         writing u, adding a refinement correction, or evaluating L u_i and
//         F_i = q + g(u_i) (eq. 9); or, instead of the solve, evaluating L u and F of a
//         given canonical vector (stage 1 uses u^n);
//   up:   the next stage right-hand side rhs = u^n + dt sum_j (a_ij L u_j + ahat_ij F_j)
//         (eq. 10) -- the newest L u_j, F_j come straight from LDS -- then
//         w = A_ii^{-1} rhs and the particular fluxes h = flux rows . w (eqs. 5-6); or the
//         interior step update u^{n+1} = u^n + dt sum_j (b_j L u_j + bhat_j F_j) and the
//         interior part of the edge fluxes for the interface-line solves.
// Everything the two phases exchange is leaf-local, so fusing them saves a launch per
// stage and overlaps the tail of one stream with the start of the next.  The FP32
// refinement passes fuse the same way: the kernel that writes u (or adds a correction)
// evaluates the FP64 residual of the new u on its tile and starts the next correction's
// solve from it, or, after a stage's last correction, evaluates L u_i, F_i and opens the
// next stage.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hps_device.h"

namespace hps {

constexpr int LPF = 2;    // operator loads issued ahead of each stream
constexpr int LUNR = 8;   // operator loads in flight in the streaming loop

// Sum the G column-group partials of `rows` rows (LDS, [g][rows]) and call fin(row, y).
// Several threads share a row; the slices are added in a fixed order (deterministic).
template <typename T, typename Fin>
__device__ __forceinline__ void reduce_rows(const T *part, int rows, int G, double *red, Fin fin) {
    for (int r0 = 0; r0 < rows; r0 += NT) {
        const int nr = min(NT, rows - r0);
        const int nsl = min(G, NT / nr);
        const int t = threadIdx.x;
        const int row = t % nr, sl = t / nr;
        if (sl < nsl) {
            T y = T(0);
            for (int gg = sl; gg < G; gg += nsl) y += part[gg * rows + r0 + row];
            red[sl * nr + row] = (double)y;
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

enum { DOWN_NONE = 0, DOWN_WRITE_U = 1, DOWN_STAGE = 2, DOWN_IR_ADD = 3, DOWN_EVAL = 4 };
// DOWN_WRITE_U / DOWN_IR_ADD followed by the refinement residual of the new u at the leaf's
// interior nodes (into LDS, where the UP_BODY phase takes it as its right-hand side) and the
// coordinate fluxes on its edges (for the interface jumps): the arithmetic of the separate
// residual evaluation, with the edge values from the leaf's own running copy of its boundary
// values (which equals u there bit for bit: both add up the same sweep outputs)
enum { DOWN_WRITE_U_RES = 5, DOWN_IR_ADD_RES = 6 };
// DOWN_IR_ADD followed by DOWN_EVAL's evaluation of L u_i and F_i on the corrected tile (the
// stage's last refinement pass fused with the phase that closes the stage)
enum { DOWN_IR_ADD_EVAL = 7 };
enum { UP_NONE = 0, UP_BODY = 1, UP_STAGE = 2, UP_UPDATE = 3 };

struct LeafArgs {
    LeafGeo geo;
    const int *leaf_ij;
    const double *D, *D2, *coef;
    int down, up;
    int xs_cap, part_cap;
    // down phase
    PanelView sl;
    const double *ub, *w_in;     // leaf boundary values [leaf][4q], particular solutions [leaf][q2]
    const double *u_eval;        // DOWN_EVAL: canonical vector evaluated
    double *u_out;               // DOWN_WRITE_U / DOWN_IR_ADD
    double *Lu_out, *F_out;      // DOWN_STAGE / DOWN_EVAL: L u_i, F_i (interior, canonical)
    const double *q_src;
    double q_scale;
    const double *q_scale_ptr;   // device scalar replacing q_scale when set
    GPoly g;
    double *norm_part;           // DOWN_IR_ADD: this leaf's max|delta|, max|u| at [2 leaf], [2 leaf + 1]
    // DOWN_*_RES: the right-hand side of the refined system, gamma dt, the leaf's running
    // boundary values [leaf][4q] and the edge fluxes (canonical leaf order) [leaf][4q]
    const double *res_rhs;
    double gamma_dt;
    double *ubc, *res_flux;
    // up phase
    PanelView ainv;
    const double *body;          // UP_BODY
    const double *un;            // UP_STAGE / UP_UPDATE: u^n (canonical)
    const double *Lu_in, *F_in;  // stage vectors [stage][n_int]
    int nprev;                   // stages before the one being assembled (the last is in LDS)
    double ca[8], cf[8];         // dt a_ij, dt ahat_ij (UP_STAGE) or dt b_j, dt bhat_j (UP_UPDATE)
    double *rhs_copy;
    double *w_out, *h_out;
    double *unew, *fpart;        // UP_UPDATE
};

__device__ __forceinline__ double poly_g(const GPoly &g, double u) {
    if (g.kind == 0) return 0.0;
    return g.g0 + u * (g.g1 + u * (g.g2 + u * g.g3));
}

// u^n + sum over the stages before `last` of (ca_j L u_j + cf_j F_j) at interior node
// base + k: the part of a stage right-hand side (or of the step update) that does not
// depend on the stage just solved, so its loads can be issued early.
__device__ __forceinline__ double older_stages(const LeafArgs &a, int64_t base, int k, int last) {
    const int64_t n_int = a.geo.n_int;
    double r = a.un[base + k];
    for (int j = 0; j < last; ++j) {
        r += a.ca[j] * a.Lu_in[j * n_int + base + k];
        r += a.cf[j] * a.F_in[j * n_int + base + k];
    }
    return r;
}

constexpr int HOIST = 1;   // interior nodes per thread whose older-stage sums are hoisted

// One leaf (heap index `leaf`) of one operator: the down phase of the stage that ends here
// and the up phase of the stage that starts here, as selected by DN and UPM.
template <typename T, int DN, int UPM>
__device__ __forceinline__ void leaf_body(const LeafArgs &a, int leaf, unsigned char *smem, double *red,
                                          double (*nred)[NT / 64]) {
    constexpr int VW = 16 / sizeof(T);
    constexpr bool res = DN == DOWN_WRITE_U_RES || DN == DOWN_IR_ADD_RES;
    constexpr bool eval_after = DN == DOWN_IR_ADD_EVAL;
    constexpr bool track = res || eval_after;   // running boundary copy, tile of the new u
    constexpr int DB = DN == DOWN_WRITE_U_RES ? DOWN_WRITE_U
                       : (DN == DOWN_IR_ADD_RES || DN == DOWN_IR_ADD_EVAL) ? DOWN_IR_ADD : DN;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q, ld = dmat_ld(p);
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int64_t n_int = a.geo.n_int;
    Carve cv{smem};
    T *xs = cv.take<T>(a.xs_cap);
    T *part = cv.take<T>(a.part_cap);
    double *tile = cv.take<double>(p * p);
    double *D = cv.take<double>(p * ld);
    double *D2 = cv.take<double>(p * ld);
    double *luv = cv.take<double>(q2);
    double *fv = cv.take<double>(q2);
    constexpr bool stream_down = DB == DOWN_WRITE_U || DB == DOWN_STAGE || DB == DOWN_IR_ADD;
    constexpr bool stream_up = UPM == UP_BODY || UPM == UP_STAGE;
    constexpr bool need_L = DB == DOWN_STAGE || DB == DOWN_EVAL;
    // the older stages' part of the next right-hand side (or of the update), loaded while the
    // down phase gathers its own inputs instead of after it
    constexpr bool hoist = (UPM == UP_STAGE || UPM == UP_UPDATE) && DB != DOWN_NONE;
    const int last_old = UPM == UP_STAGE ? a.nprev - 1 : a.nprev;
    double older[HOIST];
    auto load_older = [&]() {
        if constexpr (hoist) {
#pragma unroll
            for (int i = 0; i < HOIST; ++i) {
                const int k = threadIdx.x + i * NT;
                older[i] = k < q2 ? older_stages(a, base, k, last_old) : 0.0;
            }
        }
    };
    PanelStream<T, LPF, LUNR> ps;
    if constexpr (stream_down)
        ps.start(reinterpret_cast<const T *>(a.sl.data) + (int64_t)leaf * a.sl.node_elems, a.sl.rp, a.sl.G, a.sl.S,
                 a.sl.node_elems == 0);
    else if constexpr (stream_up)
        ps.start(reinterpret_cast<const T *>(a.ainv.data) + (int64_t)leaf * a.ainv.node_elems, a.ainv.rp, a.ainv.G,
                 a.ainv.S, a.ainv.node_elems == 0);
    load_dmat_ld(a.D, D, p);
    if (need_L || track) load_dmat_ld(a.D2, D2, p);

    // ---------------- down phase ----------------
    if constexpr (DB != DOWN_NONE) {
        // particular solution w of this leaf, staged in LDS before the stream is consumed
        if (stream_down)
            for (int k = threadIdx.x; k < q2; k += NT) fv[k] = a.w_in[(int64_t)leaf * q2 + k];
        for (int k = threadIdx.x; k < p * p; k += NT) tile[k] = 0.0;
        if constexpr (stream_down) {
            const double *ubl = a.ub + (int64_t)leaf * nb;
            const int SG = a.sl.S * a.sl.G;
            for (int k = threadIdx.x; k < SG; k += NT) xs[k] = (T)(k < nb ? ubl[k] : 0.0);
            load_older();
            __syncthreads();
            for (int k = threadIdx.x; k < nb; k += NT) tile[edge_tile_pos(p, q, k / q, k % q)] = ubl[k];
            ps.finish(xs, part);
            if constexpr (stream_up)
                ps.start(reinterpret_cast<const T *>(a.ainv.data) + (int64_t)leaf * a.ainv.node_elems, a.ainv.rp,
                         a.ainv.G, a.ainv.S, a.ainv.node_elems == 0);
            __syncthreads();
            // u_i interior = S_leaf u_b + w (this thread's rows are its own interior nodes)
            reduce_rows<T>(part, a.sl.rp * VW, a.sl.G, red, [&](int row, double y) {
                if (row < q2) tile[(row / q + 1) * p + (row % q) + 1] = y + fv[row];
            });
        } else {
            // DOWN_EVAL: the tile of a given canonical vector
            load_older();
            __syncthreads();
            for (int k = threadIdx.x; k < q2; k += NT) tile[(k / q + 1) * p + (k % q) + 1] = a.u_eval[base + k];
            for (int k = threadIdx.x; k < nb; k += NT)
                tile[edge_tile_pos(p, q, k / q, k % q)] = a.u_eval[edge_index(a.geo, li, lj, k / q, k % q)];
            __syncthreads();
        }
        // L u_i and F_i = q + g(u_i) at the interior nodes from the tile (eq. 9)
        auto eval_stage = [&]() {
            const double qs = a.q_scale_ptr ? *a.q_scale_ptr : a.q_scale;
            for (int k = threadIdx.x; k < q2; k += NT) {
                const int aa = k % q + 1, bb = k / q + 1;
                double ux = 0, uxx = 0, uy = 0, uyy = 0;
                for (int m = 0; m < p; ++m) {
                    const double xr = tile[bb * p + m];
                    const double yc = tile[m * p + aa];
                    ux = fma(D[aa * ld + m], xr, ux);
                    uxx = fma(D2[aa * ld + m], xr, uxx);
                    uy = fma(D[bb * ld + m], yc, uy);
                    uyy = fma(D2[bb * ld + m], yc, uyy);
                }
                const double u = tile[bb * p + aa];
                double cf[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) cf[c] = a.coef[c * n_int + base + k];
                const double Lu = apply_L_point(cf, uxx, uyy, ux, uy, u);
                const double F = (a.q_src ? qs * a.q_src[base + k] : 0.0) + poly_g(a.g, u);
                luv[k] = Lu;
                fv[k] = F;
                a.Lu_out[base + k] = Lu;
                a.F_out[base + k] = F;
            }
        };
        if constexpr (need_L) {
            eval_stage();
        } else if constexpr (DB == DOWN_WRITE_U || DB == DOWN_IR_ADD) {
            double dmax = 0.0, umax = 0.0;
            const double *ubl = a.ub + (int64_t)leaf * nb;
            for (int k = threadIdx.x; k < q2 + nb; k += NT) {
                int64_t gi;
                double v;
                bool own = true;
                if (k < q2) {
                    gi = base + k;
                    v = tile[(k / q + 1) * p + (k % q) + 1];
                } else {
                    const int e = (k - q2) / q, m = (k - q2) % q;
                    // each edge node is written by exactly one leaf: left/bottom edges always,
                    // right/top edges only on the last column/row of leaves
                    own = (e == 0 || e == 2) || (e == 1 && li == a.geo.n1 - 1) || (e == 3 && lj == a.geo.n2 - 1);
                    gi = edge_index(a.geo, li, lj, e, m);
                    v = ubl[k - q2];
                    if constexpr (track) {
                        // every edge node, owned or not: the leaf's running boundary value
                        double *bc = a.ubc + (int64_t)leaf * nb + (k - q2);
                        const double nbv = DB == DOWN_WRITE_U ? v : *bc + v;
                        *bc = nbv;
                        tile[edge_tile_pos(p, q, e, m)] = nbv;
                    }
                }
                if (!own) continue;
                if (DB == DOWN_WRITE_U) {
                    a.u_out[gi] = v;
                } else {
                    const double nu = a.u_out[gi] + v;
                    a.u_out[gi] = nu;
                    dmax = fmax(dmax, fabs(v));
                    umax = fmax(umax, fabs(nu));
                    if (track && k < q2) tile[(k / q + 1) * p + (k % q) + 1] = nu;
                }
            }
            if (DB == DOWN_IR_ADD) {
                for (int off = 32; off > 0; off >>= 1) {
                    dmax = fmax(dmax, __shfl_xor(dmax, off));
                    umax = fmax(umax, __shfl_xor(umax, off));
                }
                if ((threadIdx.x & 63) == 0) {
                    nred[0][threadIdx.x >> 6] = dmax;
                    nred[1][threadIdx.x >> 6] = umax;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    double dd = 0, uu = 0;
                    for (int w = 0; w < NT / 64; ++w) {
                        dd = fmax(dd, nred[0][w]);
                        uu = fmax(uu, nred[1][w]);
                    }
                    // one slot per leaf, folded by a later launch: thousands of atomics on
                    // one address serialise at the memory side
                    a.norm_part[2 * leaf] = dd;
                    a.norm_part[2 * leaf + 1] = uu;
                }
            }
        }
        __syncthreads();
        if constexpr (eval_after) {
            eval_stage();
            __syncthreads();
        }
        if constexpr (res) {
            // refinement residual rhs - (u - gamma dt L u) of the new u (into luv, the up
            // phase's right-hand side) and the edge fluxes, as the residual evaluation does
            for (int k = threadIdx.x; k < q2; k += NT) {
                const int64_t gi = base + k;
                double cf[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) cf[c] = a.coef[c * n_int + gi];
                const double rh = a.res_rhs[gi];
                const int ca = k % q + 1, cb = k / q + 1;
                double ux = 0, uxx = 0, uy = 0, uyy = 0;
                for (int m = 0; m < p; ++m) {
                    const double xr = tile[cb * p + m];
                    const double yc = tile[m * p + ca];
                    ux = fma(D[ca * ld + m], xr, ux);
                    uxx = fma(D2[ca * ld + m], xr, uxx);
                    uy = fma(D[cb * ld + m], yc, uy);
                    uyy = fma(D2[cb * ld + m], yc, uyy);
                }
                const double u = tile[cb * p + ca];
                const double Lu = apply_L_point(cf, uxx, uyy, ux, uy, u);
                luv[k] = rh - fma(-a.gamma_dt, Lu, u);
            }
            const int64_t cl = (int64_t)lj * a.geo.n1 + li;
            for (int k = threadIdx.x; k < nb; k += NT) {
                const int e = k / q, m = k % q;
                const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * ld);
                double f = 0.0;
                if (e < 2) {
                    for (int c = 0; c < p; ++c) f = fma(dr[c], tile[(m + 1) * p + c], f);
                } else {
                    for (int c = 0; c < p; ++c) f = fma(dr[c], tile[c * p + m + 1], f);
                }
                a.res_flux[cl * nb + k] = f;
            }
            __syncthreads();
        }
    }

    // ---------------- up phase ----------------
    if constexpr (UPM == UP_NONE) return;
    if constexpr (UPM == UP_UPDATE) {
        // interior u^{n+1}; the newest stage's L u, F are in LDS
        const int last = a.nprev;
        for (int k = threadIdx.x, i = 0; k < q2; k += NT, ++i) {
            double v = (hoist && i < HOIST) ? older[i] : older_stages(a, base, k, last);
            v += a.ca[last] * luv[k] + a.cf[last] * fv[k];
            a.unew[base + k] = v;
            tile[k] = v;   // reuse as the interior values, row-major
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nb; k += NT) {
            const int e = k / q, m = k % q;
            const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * ld);
            double f = 0.0;
            if (e < 2) {
                for (int c = 1; c <= q; ++c) f = fma(dr[c], tile[m * q + c - 1], f);
            } else {
                for (int c = 1; c <= q; ++c) f = fma(dr[c], tile[(c - 1) * q + m], f);
            }
            a.fpart[((int64_t)lj * a.geo.n1 + li) * nb + k] = f;
        }
        return;
    }
    const int SG = a.ainv.S * a.ainv.G;
    for (int k = threadIdx.x, i = 0; k < SG; k += NT, ++i) {
        double r = 0.0;
        if (k < q2) {
            if (UPM == UP_BODY) {
                r = res ? luv[k] : a.body[base + k];
            } else {
                const int last = a.nprev - 1;   // newest stage, held in LDS
                r = (hoist && i < HOIST) ? older[i] : older_stages(a, base, k, last);
                r += a.ca[last] * luv[k] + a.cf[last] * fv[k];
                if (a.rhs_copy) a.rhs_copy[base + k] = r;
            }
        }
        xs[k] = (T)r;
    }
    __syncthreads();
    ps.finish(xs, part);
    __syncthreads();
    double *wv = luv;   // w = A_ii^{-1} rhs; luv is free again
    reduce_rows<T>(part, a.ainv.rp * VW, a.ainv.G, red, [&](int row, double y) {
        if (row < q2) {
            wv[row] = y;
            a.w_out[(int64_t)leaf * q2 + row] = y;
        }
    });
    for (int k = threadIdx.x; k < nb; k += NT) {
        const int e = k / q, m = k % q;
        const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * ld);
        double h = 0.0;
        if (e < 2) {
            for (int c = 1; c <= q; ++c) h = fma(dr[c], wv[m * q + c - 1], h);
        } else {
            for (int c = 1; c <= q; ++c) h = fma(dr[c], wv[(c - 1) * q + m], h);
        }
        a.h_out[(int64_t)leaf * nb + k] = h;
    }
}

template <typename T, int DN, int UPM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_leaf(LeafArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT];
    __shared__ double nred[2][NT / 64];
    leaf_body<T, DN, UPM>(a, blockIdx.x, smem, red, nred);
}

// The leaves of several operators in one launch: workgroup w works on leaf w - base[b] of
// problem b, base[b] <= w < base[b + 1] (found by bisection; uniform per workgroup).
template <typename T, int DN, int UPM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_leaf_group(
    const LeafArgs *args, const int *base, int nprob) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT];
    __shared__ double nred[2][NT / 64];
    const int w = blockIdx.x;
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    leaf_body<T, DN, UPM>(args[lo], w - base[lo], smem, red, nred);
}

// =======================================================================================
// Two-component systems on one operator (the Burgers system of Sec. 5.4): one workgroup
// per leaf runs the down and up phases of both components.  Each operator block is
// streamed once and applied to both components' vectors; the explicit term couples them
// at the interior nodes:
//   F^u = q^u - (u u_x + v u_y),   F^v = q^v - (u v_x + v v_y),
// with the derivatives taken on the leaf tiles exactly as in L (eq. 3).
// =======================================================================================
struct LeafSysArgs {
    LeafArgs c[2];   // per component; the operator fields of c[0] and c[1] are the same
};

template <int DN, int UPM>
__device__ __forceinline__ void leaf_sys_body(const LeafSysArgs &A, int leaf, unsigned char *smem, double *red) {
    constexpr int NC = 2, VW = 2;
    const LeafArgs &a = A.c[0];
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q, pp = p * p;
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int64_t n_int = a.geo.n_int;
    const int xcap = a.xs_cap, pcap = a.part_cap;
    Carve cv{smem};
    double *xs = cv.take<double>((size_t)NC * xcap);
    double *part = cv.take<double>((size_t)NC * pcap);
    double *tile = cv.take<double>((size_t)NC * pp);
    const int ld = dmat_ld(p);
    double *D = cv.take<double>((size_t)p * ld);
    double *D2 = cv.take<double>((size_t)p * ld);
    double *luv = cv.take<double>((size_t)NC * q2);
    double *fv = cv.take<double>((size_t)NC * q2);
    constexpr bool stream_down = DN == DOWN_STAGE;
    PanelStream<double, LPF, LUNR> ps;
    if constexpr (stream_down)
        ps.start(reinterpret_cast<const double *>(a.sl.data) + (int64_t)leaf * a.sl.node_elems, a.sl.rp, a.sl.G, a.sl.S,
                 a.sl.node_elems == 0);
    else if constexpr (UPM == UP_STAGE)
        ps.start(reinterpret_cast<const double *>(a.ainv.data) + (int64_t)leaf * a.ainv.node_elems, a.ainv.rp,
                 a.ainv.G, a.ainv.S, a.ainv.node_elems == 0);
    load_dmat_ld(a.D, D, p);
    load_dmat_ld(a.D2, D2, p);

    // ---------------- down phase: the tiles of u_i and v_i ----------------
    for (int k = threadIdx.x; k < NC * pp; k += NT) tile[k] = 0.0;
    if constexpr (stream_down) {
        const int SG = a.sl.S * a.sl.G;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double *ubl = A.c[c].ub + (int64_t)leaf * nb;
            for (int k = threadIdx.x; k < q2; k += NT) fv[c * q2 + k] = A.c[c].w_in[(int64_t)leaf * q2 + k];
            for (int k = threadIdx.x; k < SG; k += NT) xs[c * xcap + k] = k < nb ? ubl[k] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double *ubl = A.c[c].ub + (int64_t)leaf * nb;
            for (int k = threadIdx.x; k < nb; k += NT) tile[c * pp + edge_tile_pos(p, q, k / q, k % q)] = ubl[k];
        }
        ps.finish_n<NC>(xs, xcap, part, pcap);
        if constexpr (UPM == UP_STAGE)
            ps.start(reinterpret_cast<const double *>(a.ainv.data) + (int64_t)leaf * a.ainv.node_elems, a.ainv.rp,
                     a.ainv.G, a.ainv.S, a.ainv.node_elems == 0);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c)
            reduce_rows<double>(part + c * pcap, a.sl.rp * VW, a.sl.G, red, [&](int row, double y) {
                if (row < q2) tile[c * pp + (row / q + 1) * p + (row % q) + 1] = y + fv[c * q2 + row];
            });
    } else {
        // DOWN_EVAL: the tiles of given canonical vectors
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double *ue = A.c[c].u_eval;
            for (int k = threadIdx.x; k < q2; k += NT) tile[c * pp + (k / q + 1) * p + (k % q) + 1] = ue[base + k];
            for (int k = threadIdx.x; k < nb; k += NT)
                tile[c * pp + edge_tile_pos(p, q, k / q, k % q)] = ue[edge_index(a.geo, li, lj, k / q, k % q)];
        }
        __syncthreads();
    }
    // L u_i, L v_i and the coupled advection terms
    {
        double qs[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) qs[c] = A.c[c].q_scale_ptr ? *A.c[c].q_scale_ptr : A.c[c].q_scale;
        for (int k = threadIdx.x; k < q2; k += NT) {
            const int aa = k % q + 1, bb = k / q + 1;
            const double *cf = a.coef + base + k;
            double val[NC], dx[NC], dy[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
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
                val[c] = tc[bb * p + aa];
                dx[c] = ux;
                dy[c] = uy;
                const double Lu = cf[0] * uxx + cf[n_int] * uyy + cf[2 * n_int] * ux + cf[3 * n_int] * uy +
                                  cf[4 * n_int] * val[c];
                luv[c * q2 + k] = Lu;
                A.c[c].Lu_out[base + k] = Lu;
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double src = A.c[c].q_src ? qs[c] * A.c[c].q_src[base + k] : 0.0;
                const double F = src - (val[0] * dx[c] + val[1] * dy[c]);
                fv[c * q2 + k] = F;
                A.c[c].F_out[base + k] = F;
            }
        }
    }
    __syncthreads();

    // ---------------- up phase ----------------
    if constexpr (UPM == UP_UPDATE) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const LeafArgs &ac = A.c[c];
            const int last = ac.nprev;
            double *vals = tile + c * pp;   // interior values of u^{n+1}, row-major q x q
            for (int k = threadIdx.x; k < q2; k += NT) {
                double v = ac.un[base + k];
                for (int j = 0; j < last; ++j) {
                    v += ac.ca[j] * ac.Lu_in[j * n_int + base + k];
                    v += ac.cf[j] * ac.F_in[j * n_int + base + k];
                }
                v += ac.ca[last] * luv[c * q2 + k] + ac.cf[last] * fv[c * q2 + k];
                ac.unew[base + k] = v;
                vals[k] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
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
                A.c[c].fpart[((int64_t)lj * a.geo.n1 + li) * nb + k] = f;
            }
        }
        return;
    }
    const int SG = a.ainv.S * a.ainv.G;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const LeafArgs &ac = A.c[c];
        for (int k = threadIdx.x; k < SG; k += NT) {
            double r = 0.0;
            if (k < q2) {
                r = ac.un[base + k];
                const int last = ac.nprev - 1;   // newest stage, held in LDS
                for (int j = 0; j < last; ++j) {
                    r += ac.ca[j] * ac.Lu_in[j * n_int + base + k];
                    r += ac.cf[j] * ac.F_in[j * n_int + base + k];
                }
                r += ac.ca[last] * luv[c * q2 + k] + ac.cf[last] * fv[c * q2 + k];
            }
            xs[c * xcap + k] = r;
        }
    }
    __syncthreads();
    ps.finish_n<NC>(xs, xcap, part, pcap);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double *wv = luv + c * q2;   // w = A_ii^{-1} rhs; luv is free again
        reduce_rows<double>(part + c * pcap, a.ainv.rp * VW, a.ainv.G, red, [&](int row, double y) {
            if (row < q2) {
                wv[row] = y;
                A.c[c].w_out[(int64_t)leaf * q2 + row] = y;
            }
        });
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double *wv = luv + c * q2;
        for (int k = threadIdx.x; k < nb; k += NT) {
            const int e = k / q, m = k % q;
            const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * ld);
            double h = 0.0;
            if (e < 2) {
                for (int cc = 1; cc <= q; ++cc) h = fma(dr[cc], wv[m * q + cc - 1], h);
            } else {
                for (int cc = 1; cc <= q; ++cc) h = fma(dr[cc], wv[(cc - 1) * q + m], h);
            }
            A.c[c].h_out[(int64_t)leaf * nb + k] = h;
        }
    }
}

template <int DN, int UPM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_leaf_sys(LeafSysArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT];
    leaf_sys_body<DN, UPM>(a, blockIdx.x, smem, red);
}

// =======================================================================================
// Several right-hand sides of one operator (hps_solve with nrhs > 1): one workgroup per
// leaf streams A_ii^{-1} (up: particular solutions w and fluxes h) or S_leaf (down:
// u = S_leaf u_b + w) once and applies every 16-byte load to all NC vectors.  Each
// right-hand side sees exactly the arithmetic of the single-right-hand-side kernels.
// =======================================================================================
struct LeafMultiArgs {
    LeafGeo geo;
    const int *leaf_ij;
    const double *D;
    PanelView sl, ainv;
    int xs_cap, part_cap;
    const double *body[MAX_MULTI];   // up: right-hand sides (interior, canonical)
    double *u_out[MAX_MULTI];        // down: solutions (canonical)
    const double *ub[MAX_MULTI];     // leaf boundary values [leaf][4q]
    double *w[MAX_MULTI];            // particular solutions [leaf][q2] (written up, read down)
    double *h_out[MAX_MULTI];        // particular fluxes [leaf][4q]
};

template <int NC, bool UP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_leaf_multi(LeafMultiArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT];
    constexpr int VW = 2;
    const int leaf = blockIdx.x;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q;
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    Carve cv{smem};
    double *xs = cv.take<double>((size_t)NC * a.xs_cap);
    double *part = cv.take<double>((size_t)NC * a.part_cap);
    double *D = cv.take<double>(p * p);
    double *wv = cv.take<double>((size_t)NC * q2);
    const PanelView &pv = UP ? a.ainv : a.sl;
    PanelStream<double, LPF, LUNR> ps;
    ps.start(reinterpret_cast<const double *>(pv.data) + (int64_t)leaf * pv.node_elems, pv.rp, pv.G, pv.S,
             pv.node_elems == 0);
    load_dmat(a.D, D, p * p);
    const int SG = pv.S * pv.G, pst = pv.G * pv.rp * VW, rows = pv.rp * VW;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        for (int k = threadIdx.x; k < SG; k += NT) {
            double x = 0.0;
            if (UP) x = k < q2 ? a.body[c][base + k] : 0.0;
            else x = k < nb ? a.ub[c][(int64_t)leaf * nb + k] : 0.0;
            xs[c * SG + k] = x;
        }
        if (!UP)
            for (int k = threadIdx.x; k < q2; k += NT) wv[c * q2 + k] = a.w[c][(int64_t)leaf * q2 + k];
    }
    __syncthreads();
    ps.finish_n<NC>(xs, SG, part, pst);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        reduce_rows<double>(part + c * pst, rows, pv.G, red, [&](int row, double y) {
            if (row >= q2) return;
            if (UP) {
                wv[c * q2 + row] = y;
                a.w[c][(int64_t)leaf * q2 + row] = y;
            } else {
                a.u_out[c][base + row] = y + wv[c * q2 + row];
            }
        });
    }
    if (UP) {
        // particular fluxes h = flux rows . w (the interior part of the edge derivative)
        for (int idx = threadIdx.x; idx < NC * nb; idx += NT) {
            const int c = idx / nb, k = idx - c * nb;
            const int e = k / q, m = k % q;
            const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * p);
            const double *w = wv + c * q2;
            double h = 0.0;
            if (e < 2) {
                for (int cc = 1; cc <= q; ++cc) h = fma(dr[cc], w[m * q + cc - 1], h);
            } else {
                for (int cc = 1; cc <= q; ++cc) h = fma(dr[cc], w[(cc - 1) * q + m], h);
            }
            a.h_out[c][(int64_t)leaf * nb + k] = h;
        }
    } else {
        // edge values: each edge node is written by exactly one leaf (left / bottom edges
        // always, right / top edges only on the last column / row of leaves)
        for (int idx = threadIdx.x; idx < NC * nb; idx += NT) {
            const int c = idx / nb, k = idx - c * nb;
            const int e = k / q, m = k % q;
            const bool own = (e == 0 || e == 2) || (e == 1 && li == a.geo.n1 - 1) || (e == 3 && lj == a.geo.n2 - 1);
            if (own) a.u_out[c][edge_index(a.geo, li, lj, e, m)] = a.ub[c][(int64_t)leaf * nb + k];
        }
    }
}

// =======================================================================================
// launcher
// =======================================================================================
static int leaf_family(const LeafPhase &ph, bool fp32) {
    const bool stage_down = ph.down == LD_STAGE;
    if (ph.down == LD_EVAL) return ph.up == LU_UPDATE ? KF_LEAF_EVAL_UPDATE64 : (fp32 ? KF_LEAF_EVAL_UP32 : KF_LEAF_EVAL_UP64);
    if (stage_down && ph.up == LU_UPDATE) return KF_LEAF_DOWN_UPDATE64;
    if (stage_down) return fp32 ? KF_LEAF_DOWN_UP32 : KF_LEAF_DOWN_UP64;
    if (ph.down != LD_NONE) return fp32 ? KF_LEAF_DOWN32 : KF_LEAF_DOWN64;
    return fp32 ? KF_LEAF_UP32 : KF_LEAF_UP64;
}

static void make_leaf_args(const hps_op *op, bool fp32, const LeafPhase &ph, LeafArgs &a, size_t &lds) {
    a = LeafArgs{};
    a.geo = geo_of(op);
    a.leaf_ij = op->leaf_ij;
    a.D = op->D;
    a.D2 = op->D2;
    a.coef = op->coef;
    a.down = ph.down;
    a.up = ph.up;
    const Panel &sl = fp32 ? op->sleaf32 : op->sleaf64;
    const Panel &ai = fp32 ? op->ainv32 : op->ainv64;
    a.sl = view(sl);
    a.ainv = view(ai);
    const int vw = fp32 ? 4 : 2;
    a.xs_cap = std::max(sl.S * sl.G, ai.S * ai.G);
    a.part_cap = std::max(sl.G * sl.rp, ai.G * ai.rp) * vw;
    a.ub = op->ub_leaf;
    a.w_in = op->w_leaf;
    a.u_eval = ph.u_eval;
    a.u_out = ph.u_out;
    a.Lu_out = ph.Lu_out;
    a.F_out = ph.F_out;
    a.q_src = ph.q_src;
    a.q_scale = ph.q_scale;
    a.q_scale_ptr = ph.q_scale_ptr;
    a.g = ph.g;
    a.norm_part = ph.norm_part ? ph.norm_part : op->ir_part;
    a.res_rhs = ph.res_rhs;
    a.gamma_dt = op->gamma_dt;
    a.ubc = op->ir_ubc;
    a.res_flux = op->ir_flux;
    a.body = ph.body;
    a.un = ph.un;
    a.Lu_in = ph.Lu_in;
    a.F_in = ph.F_in;
    a.nprev = ph.nprev;
    for (int j = 0; j < 8; ++j) {
        a.ca[j] = ph.ca[j];
        a.cf[j] = ph.cf[j];
    }
    a.rhs_copy = ph.rhs_copy;
    a.w_out = op->w_leaf;
    a.h_out = op->h_leaf;
    a.unew = ph.unew;
    a.fpart = op->ir_flux;
    const size_t es = fp32 ? 4 : 8;
    const size_t pp = (size_t)op->p * op->p * 8, pd = (size_t)op->p * dmat_ld(op->p) * 8, q2b = (size_t)op->q2 * 8;
    lds = carve_bytes({(size_t)a.xs_cap * es, (size_t)a.part_cap * es, pp, pd, pd, q2b, q2b});
}

static void use_leaf_workspace(LeafArgs &a, const Workspace *ws) {
    if (!ws) return;
    a.ub = ws->ub_leaf;
    a.w_in = ws->w_leaf;
    a.w_out = ws->w_leaf;
    a.h_out = ws->h_leaf;
    a.fpart = ws->flux;
    a.res_flux = ws->flux;
    a.ubc = ws->ir_ubc;
}

int leaf_kernel_mode(const LeafPhase &ph, bool fp32) {
    if (fp32 && ph.ir_eval && ph.down == LD_IR_ADD && (ph.up == LU_STAGE || ph.up == LU_UPDATE)) return DOWN_IR_ADD_EVAL;
    if (fp32 && ph.res_rhs && ph.up == LU_BODY) {
        if (ph.down == LD_WRITE_U) return DOWN_WRITE_U_RES;
        if (ph.down == LD_IR_ADD) return DOWN_IR_ADD_RES;
    }
    return ph.down;
}

int launch_leaf(const hps_op *op, bool fp32, const LeafPhase &ph, hipStream_t st, const Workspace *ws) {
    ProfScope ps_(&op->prof, leaf_family(ph, fp32), st);
    LeafArgs a;
    size_t lds = 0;
    make_leaf_args(op, fp32, ph, a, lds);
    use_leaf_workspace(a, ws);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(op->nleaves), dim3(NT), lds, st, a); };
#define HPS_LEAF_CASE(DNV, UPV)                                                   \
    if (ph.down == DNV && ph.up == UPV) {                                         \
        if (fp32) go(k_leaf<float, DNV, UPV>);                                    \
        else go(k_leaf<double, DNV, UPV>);                                        \
        HPS_LAUNCHED();                                                           \
        return HPS_OK;                                                            \
    }
    HPS_LEAF_CASE(DOWN_EVAL, UP_STAGE)
    HPS_LEAF_CASE(DOWN_STAGE, UP_STAGE)
    HPS_LEAF_CASE(DOWN_STAGE, UP_UPDATE)
    HPS_LEAF_CASE(DOWN_EVAL, UP_UPDATE)
    HPS_LEAF_CASE(DOWN_NONE, UP_BODY)
    HPS_LEAF_CASE(DOWN_WRITE_U, UP_NONE)
    HPS_LEAF_CASE(DOWN_IR_ADD, UP_NONE)
#undef HPS_LEAF_CASE
    if (ph.ir_eval && fp32 && ph.down == LD_IR_ADD && (ph.up == LU_STAGE || ph.up == LU_UPDATE)) {
        if (ph.up == LU_STAGE) go(k_leaf<float, DOWN_IR_ADD_EVAL, UP_STAGE>);
        else go(k_leaf<float, DOWN_IR_ADD_EVAL, UP_UPDATE>);
        HPS_LAUNCHED();
        return HPS_OK;
    }
    if (ph.res_rhs && fp32 && ph.up == LU_BODY && (ph.down == LD_WRITE_U || ph.down == LD_IR_ADD)) {
        if (ph.down == LD_WRITE_U) go(k_leaf<float, DOWN_WRITE_U_RES, UP_BODY>);
        else go(k_leaf<float, DOWN_IR_ADD_RES, UP_BODY>);
        HPS_LAUNCHED();
        return HPS_OK;
    }
    hps_set_error("internal: unsupported leaf phase combination (%d, %d)", ph.down, ph.up);
    return HPS_EINVAL;
}

int launch_leaf_multi(const hps_op *op, int nc, bool up, const double *const *body, double *const *u,
                      const Workspace *const *ws, hipStream_t st) {
    ProfScope ps_(&op->prof, up ? KF_LEAF_UP64 : KF_LEAF_DOWN64, st);
    LeafMultiArgs a{};
    a.geo = geo_of(op);
    a.leaf_ij = op->leaf_ij;
    a.D = op->D;
    a.sl = view(op->sleaf64);
    a.ainv = view(op->ainv64);
    a.xs_cap = std::max(op->sleaf64.S * op->sleaf64.G, op->ainv64.S * op->ainv64.G);
    a.part_cap = std::max(op->sleaf64.G * op->sleaf64.rp, op->ainv64.G * op->ainv64.rp) * 2;
    for (int c = 0; c < nc; ++c) {
        const Workspace *w = ws[c];
        a.body[c] = body ? body[c] : nullptr;
        a.u_out[c] = u ? u[c] : nullptr;
        a.ub[c] = w ? w->ub_leaf : op->ub_leaf;
        a.w[c] = w ? w->w_leaf : op->w_leaf;
        a.h_out[c] = w ? w->h_leaf : op->h_leaf;
    }
    const size_t lds = carve_bytes({(size_t)nc * a.xs_cap * 8, (size_t)nc * a.part_cap * 8, (size_t)op->p * op->p * 8,
                                    (size_t)nc * op->q2 * 8});
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(op->nleaves), dim3(NT), lds, st, a); };
    switch (nc * 2 + (up ? 1 : 0)) {
        case 5: go(k_leaf_multi<2, true>); break;
        case 4: go(k_leaf_multi<2, false>); break;
        case 7: go(k_leaf_multi<3, true>); break;
        case 6: go(k_leaf_multi<3, false>); break;
        case 9: go(k_leaf_multi<4, true>); break;
        case 8: go(k_leaf_multi<4, false>); break;
        default: hps_set_error("internal: %d right-hand sides per leaf launch", nc); return HPS_EINVAL;
    }
    HPS_LAUNCHED();
    return HPS_OK;
}

size_t leaf_args_size() { return sizeof(LeafArgs); }

int fill_leaf_args(const hps_op *op, const LeafPhase &ph, void *dst, size_t *lds, const Workspace *ws, bool fp32) {
    LeafArgs &a = *reinterpret_cast<LeafArgs *>(dst);
    make_leaf_args(op, fp32, ph, a, *lds);
    use_leaf_workspace(a, ws);
    return HPS_OK;
}

int launch_leaf_group(const void *args, const int *base, int nprob, int total, size_t lds, int down, int up,
                      hipStream_t st, bool fp32) {
    if (total <= 0) return HPS_OK;
    const LeafArgs *a = reinterpret_cast<const LeafArgs *>(args);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(total), dim3(NT), lds, st, a, base, nprob); };
#define HPS_LEAF_GROUP_CASE(T, DNV, UPV)                                            \
    if (down == DNV && up == UPV) {                                                 \
        go(k_leaf_group<T, DNV, UPV>);                                              \
        HPS_LAUNCHED();                                                             \
        return HPS_OK;                                                              \
    }
    if (!fp32) {
        HPS_LEAF_GROUP_CASE(double, DOWN_EVAL, UP_STAGE)
        HPS_LEAF_GROUP_CASE(double, DOWN_STAGE, UP_STAGE)
        HPS_LEAF_GROUP_CASE(double, DOWN_STAGE, UP_UPDATE)
    } else {   // the phases of a refined FP32 step
        HPS_LEAF_GROUP_CASE(float, DOWN_EVAL, UP_STAGE)
        HPS_LEAF_GROUP_CASE(float, DOWN_EVAL, UP_UPDATE)
        HPS_LEAF_GROUP_CASE(float, DOWN_WRITE_U, UP_NONE)
        HPS_LEAF_GROUP_CASE(float, DOWN_NONE, UP_BODY)
        HPS_LEAF_GROUP_CASE(float, DOWN_IR_ADD, UP_NONE)
        HPS_LEAF_GROUP_CASE(float, DOWN_WRITE_U_RES, UP_BODY)
        HPS_LEAF_GROUP_CASE(float, DOWN_IR_ADD_RES, UP_BODY)
        HPS_LEAF_GROUP_CASE(float, DOWN_IR_ADD_EVAL, UP_STAGE)
        HPS_LEAF_GROUP_CASE(float, DOWN_IR_ADD_EVAL, UP_UPDATE)
    }
#undef HPS_LEAF_GROUP_CASE
    hps_set_error("internal: unsupported grouped leaf phase (%d, %d)", down, up);
    return HPS_EINVAL;
}

// Both components of a two-component step phase in one launch (FP64; the phase pairs of
// the stage formulation).  ws[c] redirects component c's solve buffers (null: the
// operator's own).
int launch_leaf_sys(const hps_op *op, const LeafPhase &ph0, const LeafPhase &ph1, const Workspace *ws0,
                    const Workspace *ws1, hipStream_t st) {
    ProfScope ps_(&op->prof,
                  ph0.down == LD_EVAL ? KF_LEAF2_EVAL_UP64 : (ph0.up == LU_UPDATE ? KF_LEAF2_DOWN_UPDATE64 : KF_LEAF2_DOWN_UP64),
                  st);
    LeafSysArgs A;
    size_t l0 = 0, l1 = 0;
    TRY(fill_leaf_args(op, ph0, &A.c[0], &l0, ws0));
    TRY(fill_leaf_args(op, ph1, &A.c[1], &l1, ws1));
    const size_t pp = (size_t)op->p * op->p * 8, pd = (size_t)op->p * dmat_ld(op->p) * 8, q2b = (size_t)op->q2 * 8;
    const size_t lds = carve_bytes({2 * (size_t)A.c[0].xs_cap * 8, 2 * (size_t)A.c[0].part_cap * 8, 2 * pp, pd, pd,
                                    2 * q2b, 2 * q2b});
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(op->nleaves), dim3(NT), lds, st, A); };
    if (ph0.down != ph1.down || ph0.up != ph1.up) {
        hps_set_error("internal: the two components must run the same phase");
        return HPS_EINVAL;
    }
#define HPS_LEAF_SYS_CASE(DNV, UPV)     \
    if (ph0.down == DNV && ph0.up == UPV) { \
        go(k_leaf_sys<DNV, UPV>);       \
        HPS_LAUNCHED();                 \
        return HPS_OK;                  \
    }
    HPS_LEAF_SYS_CASE(DOWN_EVAL, UP_STAGE)
    HPS_LEAF_SYS_CASE(DOWN_STAGE, UP_STAGE)
    HPS_LEAF_SYS_CASE(DOWN_STAGE, UP_UPDATE)
#undef HPS_LEAF_SYS_CASE
    hps_set_error("internal: unsupported two-component leaf phase (%d, %d)", ph0.down, ph0.up);
    return HPS_EINVAL;
}

}  // namespace hps
