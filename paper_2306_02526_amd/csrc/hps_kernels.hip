// HIP kernels of the RKHPS per-stage solve and of the HPS build, written for gfx950.
//
// Method: Chen, Appelo, Babb & Martinsson, arXiv 2306.02526.
//   Sec. 2.1 eqs. (5)-(6): leaf operators;  merge formulas after eqs. (7)-(8);
//   Algorithm 1 (solve stage) extended by the particular-solution (body load) terms;
//   Sec. 3.1 eqs. (9)-(11): stage right-hand sides and boundary data.
//
// Every solve-phase kernel streams a packed operator (struct Panel) from HBM exactly once:
// the storage order equals the order in which the workgroup's lanes read it, so each
// iteration of a workgroup is one contiguous run of 16-byte loads.  Field data (stage
// vectors, boundary data) are small next to the operators and are gathered directly.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hps_internal.h"

namespace hps {

// =======================================================================================
// streaming matrix-vector core
// =======================================================================================
template <typename T> struct V16;
template <> struct V16<double> { using type = double2; };
template <> struct V16<float> { using type = float4; };

__device__ __forceinline__ void vfma(double *acc, const double2 &v, double x) {
    acc[0] = fma(v.x, x, acc[0]);
    acc[1] = fma(v.y, x, acc[1]);
}
__device__ __forceinline__ void vfma(float *acc, const float4 &v, float x) {
    acc[0] = fmaf(v.x, x, acc[0]);
    acc[1] = fmaf(v.y, x, acc[1]);
    acc[2] = fmaf(v.z, x, acc[2]);
    acc[3] = fmaf(v.w, x, acc[3]);
}

// Accumulate one (tile, chunk) block of a Panel against xs (chunk-local, S*G entries in
// LDS, zero padded) into part[g][rp*VW] (LDS).  Caller synchronises before and after.
template <typename T>
__device__ __forceinline__ void panel_accum(const T *__restrict__ blk, int rp, int G, int S,
                                            const T *__restrict__ xs, T *__restrict__ part) {
    using V = typename V16<T>::type;
    constexpr int VW = 16 / sizeof(T);
    const int t = threadIdx.x;
    const int act = rp * G;
    if (t >= act) return;
    const int g = t / rp;
    const int r = t - g * rp;
    const V *p = reinterpret_cast<const V *>(blk) + t;
    T acc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = T(0);
    int s = 0;
    for (; s + 8 <= S; s += 8) {
        V vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vv[u] = p[(size_t)(s + u) * act];
#pragma unroll
        for (int u = 0; u < 8; ++u) vfma(acc, vv[u], xs[(s + u) * G + g]);
    }
    for (; s < S; ++s) vfma(acc, p[(size_t)s * act], xs[s * G + g]);
    T *dst = part + g * (rp * VW) + r * VW;
#pragma unroll
    for (int v = 0; v < VW; ++v) dst[v] = acc[v];
}

template <typename T>
__device__ __forceinline__ double panel_sum(const T *__restrict__ part, int rp, int G, int idx) {
    constexpr int VW = 16 / sizeof(T);
    T s = T(0);
    for (int g = 0; g < G; ++g) s += part[g * (rp * VW) + idx];
    return (double)s;
}

struct PanelView {
    const void *data;
    int rp, G, S, ntile, kch;
    int64_t tile_elems, node_elems;
};

static PanelView view(const Panel &p) {
    return PanelView{p.data, p.rp, p.G, p.S, p.ntile, p.kch, p.tile_elems, p.node_elems};
}

constexpr int XS_MAX = 1024;   // LDS capacity for the chunk-local input vector
constexpr int PART_MAX = 1024; // LDS capacity for the per-group partial sums (T elements)

// =======================================================================================
// leaf geometry helpers
// =======================================================================================
struct LeafGeo {
    int n1, n2, q, p;
    int64_t n_int, n_vert;
};

// canonical index of a leaf-edge node: e = 0 left, 1 right, 2 bottom, 3 top; m in 0..q-1
__device__ __forceinline__ int64_t edge_index(const LeafGeo &g, int i, int j, int e, int m) {
    switch (e) {
        case 0: return g.n_int + ((int64_t)i * g.n2 + j) * g.q + m;
        case 1: return g.n_int + ((int64_t)(i + 1) * g.n2 + j) * g.q + m;
        case 2: return g.n_int + g.n_vert + ((int64_t)j * g.n1 + i) * g.q + m;
        default: return g.n_int + g.n_vert + ((int64_t)(j + 1) * g.n1 + i) * g.q + m;
    }
}

// position in the p x p tile (tile[b*p + a]) of leaf-boundary entry e*q + m
__device__ __forceinline__ int edge_tile_pos(int p, int q, int e, int m) {
    switch (e) {
        case 0: return (m + 1) * p;
        case 1: return (m + 1) * p + (p - 1);
        case 2: return m + 1;
        default: return (p - 1) * p + m + 1;
    }
}

__device__ __forceinline__ void load_dmat(const double *src, double *dst, int n) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
}

// L u at interior node k of the tile: cxx u_xx + cyy u_yy + cx u_x + cy u_y + c0 u (eq. 3
// written for L, c12 = 0), derivatives along the tile row / column through the node.
__device__ __forceinline__ double tile_L(const double *tile, const double *D, const double *D2,
                                         int p, int q, const double *coef, int64_t n_int,
                                         int64_t gidx, int k) {
    const int a = k % q + 1;
    const int b = k / q + 1;
    double ux = 0, uxx = 0, uy = 0, uyy = 0;
    for (int m = 0; m < p; ++m) {
        const double xr = tile[b * p + m];
        const double yc = tile[m * p + a];
        ux = fma(D[a * p + m], xr, ux);
        uxx = fma(D2[a * p + m], xr, uxx);
        uy = fma(D[b * p + m], yc, uy);
        uyy = fma(D2[b * p + m], yc, uyy);
    }
    const double u = tile[b * p + a];
    return coef[gidx] * uxx + coef[n_int + gidx] * uyy + coef[2 * n_int + gidx] * ux +
           coef[3 * n_int + gidx] * uy + coef[4 * n_int + gidx] * u;
}

__device__ __forceinline__ double gpoly(const GPoly &g, double u) {
    if (g.kind == 0) return 0.0;
    return g.g0 + u * (g.g1 + u * (g.g2 + u * g.g3));
}

// =======================================================================================
// leaf upward kernel: stage right-hand side, w = A_ii^{-1} rhs, particular fluxes h
// =======================================================================================
struct LeafUpArgs {
    PanelView ainv;
    const int *leaf_ij;
    LeafGeo geo;
    const double *body;   // mode body: canonical interior rhs
    const double *un;     // mode stage: u^n (canonical, interior part used)
    const double *Lu, *F; // stage vectors, j-th at + j*n_int
    StageCoefs sc;
    double *rhs_copy;     // optional copy of the assembled rhs (canonical interior)
    const double *D;
    double *w_out, *h_out;
};

template <typename T>
__global__ __launch_bounds__(NT) void k_leaf_up(LeafUpArgs a) {
    constexpr int VW = 16 / sizeof(T);
    __shared__ T xs[XS_MAX];
    __shared__ T part[PART_MAX];
    __shared__ double wv[PMAX * PMAX];
    __shared__ double d0[PMAX], dl[PMAX];
    const int leaf = blockIdx.x;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q;
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int SG = a.ainv.S * a.ainv.G;
    for (int k = threadIdx.x; k < SG; k += NT) {
        double r = 0.0;
        if (k < q2) {
            if (a.body) {
                r = a.body[base + k];
            } else {
                r = a.un[base + k];
                for (int j = 0; j < a.sc.nprev; ++j) {
                    r += a.sc.ca[j] * a.Lu[j * a.geo.n_int + base + k];
                    r += a.sc.cf[j] * a.F[j * a.geo.n_int + base + k];
                }
                if (a.rhs_copy) a.rhs_copy[base + k] = r;
            }
        }
        xs[k] = (T)r;
    }
    for (int k = threadIdx.x; k < p; k += NT) {
        d0[k] = a.D[k];
        dl[k] = a.D[(p - 1) * p + k];
    }
    __syncthreads();
    panel_accum<T>(reinterpret_cast<const T *>(a.ainv.data) + (int64_t)leaf * a.ainv.node_elems,
                   a.ainv.rp, a.ainv.G, a.ainv.S, xs, part);
    __syncthreads();
    for (int k = threadIdx.x; k < q2; k += NT) {
        const double w = panel_sum<T>(part, a.ainv.rp, a.ainv.G, k);
        wv[k] = w;
        a.w_out[(int64_t)leaf * q2 + k] = w;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 4 * q; k += NT) {
        const int e = k / q, m = k - (k / q) * q;
        const double *dr = (e == 0 || e == 2) ? d0 : dl;
        double h = 0.0;
        if (e < 2) {
            for (int c = 1; c <= q; ++c) h = fma(dr[c], wv[m * q + c - 1], h);
        } else {
            for (int c = 1; c <= q; ++c) h = fma(dr[c], wv[(c - 1) * q + m], h);
        }
        a.h_out[(int64_t)leaf * 4 * q + k] = h;
    }
}

// =======================================================================================
// level kernels (upward: w3 = X d, h = [h1; h2] + U d; downward: u3 = S u12 + w3)
// =======================================================================================
struct LevelArgs {
    PanelView pn;
    int n1, n2, n3, n12, nbc;
    const int *a1, *a3, *b2, *b3;
    // upward
    const double *hc;      // children fluxes [2*nodes][nbc]
    const double *r3;      // interface jump data (interface-indexed) or null
    const int *j3i;
    double *w3, *h;
    // downward
    const double *ub;      // this level's boundary values [nodes][n12] (null at root)
    const double *dir;     // root: Dirichlet data (boundary-indexed) or null
    const int *root_map;
    double *ubc;           // children boundary values [2*nodes][nbc]
    double *part;          // split-K partials [nodes][ntile][kch][rp*vw]
    int root;
};

__device__ __forceinline__ void up_finalize(const LevelArgs &a, int node, int row, double y) {
    if (row < a.n3) {
        a.w3[(int64_t)node * a.n3 + row] = y;
    } else if (row < a.n3 + a.n12 && !a.root) {
        const int m = row - a.n3;
        const double *ha = a.hc + (int64_t)(2 * node) * a.nbc;
        const double *hb = a.hc + (int64_t)(2 * node + 1) * a.nbc;
        const double base = (m < a.n1) ? ha[a.a1[m]] : hb[a.b2[m - a.n1]];
        a.h[(int64_t)node * a.n12 + m] = base + y;
    }
}

__device__ __forceinline__ void down_finalize(const LevelArgs &a, int node, int row, double y) {
    if (row < a.n3) {
        const double u3 = y + a.w3[(int64_t)node * a.n3 + row];
        a.ubc[(int64_t)(2 * node) * a.nbc + a.a3[row]] = u3;
        a.ubc[(int64_t)(2 * node + 1) * a.nbc + a.b3[row]] = u3;
    }
}

__device__ __forceinline__ double down_input(const LevelArgs &a, int node, int k) {
    if (a.root) return a.dir ? a.dir[a.root_map[k]] : 0.0;
    return a.ub[(int64_t)node * a.n12 + k];
}

template <typename T, bool UP>
__global__ __launch_bounds__(NT) void k_level(LevelArgs a) {
    constexpr int VW = 16 / sizeof(T);
    __shared__ T xs[XS_MAX];
    __shared__ T part[PART_MAX];
    const int kch = a.pn.kch, ntile = a.pn.ntile;
    const int chunk = blockIdx.x % kch;
    const int tile = (blockIdx.x / kch) % ntile;
    const int node = blockIdx.x / (kch * ntile);
    const int SG = a.pn.S * a.pn.G;
    const int cols = UP ? a.n3 : a.n12;
    for (int k = threadIdx.x; k < SG; k += NT) {
        const int kg = chunk * SG + k;
        double x = 0.0;
        if (kg < cols) {
            if (UP) {
                const double *ha = a.hc + (int64_t)(2 * node) * a.nbc;
                const double *hb = a.hc + (int64_t)(2 * node + 1) * a.nbc;
                x = hb[a.b3[kg]] - ha[a.a3[kg]];
                if (a.r3) x += a.r3[a.j3i[(int64_t)node * a.n3 + kg]];
            } else {
                x = down_input(a, node, kg);
            }
        }
        xs[k] = (T)x;
    }
    if (!UP && tile == 0 && chunk == 0) {
        // the J1 / J2 parts of the children's boundary data are the parent's own
        for (int m = threadIdx.x; m < a.n12; m += NT) {
            const double v = down_input(a, node, m);
            if (m < a.n1) a.ubc[(int64_t)(2 * node) * a.nbc + a.a1[m]] = v;
            else a.ubc[(int64_t)(2 * node + 1) * a.nbc + a.b2[m - a.n1]] = v;
        }
    }
    __syncthreads();
    const T *blk = reinterpret_cast<const T *>(a.pn.data) + (int64_t)node * a.pn.node_elems +
                   (int64_t)(tile * kch + chunk) * a.pn.tile_elems;
    panel_accum<T>(blk, a.pn.rp, a.pn.G, a.pn.S, xs, part);
    __syncthreads();
    const int rows = a.pn.rp * VW;
    for (int idx = threadIdx.x; idx < rows; idx += NT) {
        const double y = panel_sum<T>(part, a.pn.rp, a.pn.G, idx);
        const int row = tile * rows + idx;
        if (kch == 1) {
            if (UP) up_finalize(a, node, row, y);
            else down_finalize(a, node, row, y);
        } else {
            a.part[(((int64_t)node * ntile + tile) * kch + chunk) * rows + idx] = y;
        }
    }
}

template <bool UP>
__global__ __launch_bounds__(NT) void k_level_finalize(LevelArgs a, int vw) {
    const int kch = a.pn.kch, ntile = a.pn.ntile;
    const int tile = blockIdx.x % ntile;
    const int node = blockIdx.x / ntile;
    const int rows = a.pn.rp * vw;
    for (int idx = threadIdx.x; idx < rows; idx += NT) {
        double y = 0.0;
        const double *pp = a.part + ((int64_t)node * ntile + tile) * kch * rows + idx;
        for (int c = 0; c < kch; ++c) y += pp[(int64_t)c * rows];
        const int row = tile * rows + idx;
        if (UP) up_finalize(a, node, row, y);
        else down_finalize(a, node, row, y);
    }
}

// =======================================================================================
// leaf downward kernel: u_i = S_leaf u_b + w, then (mode) write u, or L u and F, or add a
// refinement correction
// =======================================================================================
struct LeafDownArgs {
    PanelView sl;
    const int *leaf_ij;
    LeafGeo geo;
    const double *ub, *w;
    const double *D, *D2, *coef;
    int mode;
    double *u;
    double *Lu, *F;
    const double *q_src;
    double q_scale;
    GPoly g;
    unsigned long long *norms;  // mode 2: [0] max|delta|, [1] max|u| as ordered bit patterns
};

__device__ __forceinline__ void atomic_max_abs(unsigned long long *dst, double v) {
    // non-negative doubles order like their bit patterns
    atomicMax(dst, (unsigned long long)__double_as_longlong(fabs(v)));
}

template <typename T>
__global__ __launch_bounds__(NT) void k_leaf_down(LeafDownArgs a) {
    __shared__ T xs[XS_MAX];
    __shared__ T part[PART_MAX];
    __shared__ double tile[PMAX * PMAX];
    __shared__ double D[PMAX * PMAX], D2[PMAX * PMAX];
    __shared__ double red[2][NT / 64];
    const int leaf = blockIdx.x;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q;
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int SG = a.sl.S * a.sl.G;
    const double *ubl = a.ub + (int64_t)leaf * nb;
    for (int k = threadIdx.x; k < SG; k += NT) xs[k] = (T)(k < nb ? ubl[k] : 0.0);
    for (int k = threadIdx.x; k < p * p; k += NT) tile[k] = 0.0;
    if (a.mode == 1) {
        load_dmat(a.D, D, p * p);
        load_dmat(a.D2, D2, p * p);
    }
    __syncthreads();
    panel_accum<T>(reinterpret_cast<const T *>(a.sl.data) + (int64_t)leaf * a.sl.node_elems,
                   a.sl.rp, a.sl.G, a.sl.S, xs, part);
    __syncthreads();
    for (int k = threadIdx.x; k < q2; k += NT) {
        const double v = panel_sum<T>(part, a.sl.rp, a.sl.G, k) + a.w[(int64_t)leaf * q2 + k];
        tile[(k / q + 1) * p + (k % q) + 1] = v;
    }
    for (int k = threadIdx.x; k < nb; k += NT) tile[edge_tile_pos(p, q, k / q, k % q)] = ubl[k];
    __syncthreads();
    if (a.mode == 0 || a.mode == 2) {
        double dmax = 0.0, umax = 0.0;
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
                own = (e == 0 || e == 2) || (e == 1 && li == a.geo.n1 - 1) ||
                      (e == 3 && lj == a.geo.n2 - 1);
                gi = edge_index(a.geo, li, lj, e, m);
                v = ubl[k - q2];
            }
            if (!own) continue;
            if (a.mode == 0) {
                a.u[gi] = v;
            } else {
                const double nu = a.u[gi] + v;
                a.u[gi] = nu;
                dmax = fmax(dmax, fabs(v));
                umax = fmax(umax, fabs(nu));
            }
        }
        if (a.mode == 2) {
            for (int off = 32; off > 0; off >>= 1) {
                dmax = fmax(dmax, __shfl_xor(dmax, off));
                umax = fmax(umax, __shfl_xor(umax, off));
            }
            if ((threadIdx.x & 63) == 0) {
                red[0][threadIdx.x >> 6] = dmax;
                red[1][threadIdx.x >> 6] = umax;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double d = 0, uu = 0;
                for (int w = 0; w < NT / 64; ++w) {
                    d = fmax(d, red[0][w]);
                    uu = fmax(uu, red[1][w]);
                }
                atomic_max_abs(&a.norms[0], d);
                atomic_max_abs(&a.norms[1], uu);
            }
        }
        return;
    }
    // mode 1: L u_i and F_i = q + g(u_i) at the interior nodes
    for (int k = threadIdx.x; k < q2; k += NT) {
        const int64_t gi = base + k;
        a.Lu[gi] = tile_L(tile, D, D2, p, q, a.coef, a.geo.n_int, gi, k);
        const double u = tile[(k / q + 1) * p + (k % q) + 1];
        const double qv = a.q_src ? a.q_scale * a.q_src[gi] : 0.0;
        a.F[gi] = qv + gpoly(a.g, u);
    }
}

// =======================================================================================
// stage-1 evaluation (L u^n, F_1) and the refinement residual, from a canonical vector
// =======================================================================================
__device__ void tile_from_canonical(const LeafGeo &g, int li, int lj, const double *u,
                                    double *tile) {
    const int q = g.q, p = g.p, q2 = q * q;
    const int64_t base = ((int64_t)lj * g.n1 + li) * q2;
    for (int k = threadIdx.x; k < p * p; k += NT) tile[k] = 0.0;
    __syncthreads();
    for (int k = threadIdx.x; k < q2; k += NT) tile[(k / q + 1) * p + (k % q) + 1] = u[base + k];
    for (int k = threadIdx.x; k < 4 * q; k += NT) {
        const int e = k / q, m = k % q;
        tile[edge_tile_pos(p, q, e, m)] = u[edge_index(g, li, lj, e, m)];
    }
    __syncthreads();
}

struct EvalArgs {
    LeafGeo geo;
    const double *u;
    const double *D, *D2, *coef;
    double *Lu, *F;
    const double *q_src;
    double q_scale;
    GPoly g;
    // residual mode
    const double *rhs;
    double gamma_dt;
    double *r_int, *flux;
};

// one workgroup per leaf in canonical order (blockIdx.x = j*n1 + i)
__global__ __launch_bounds__(NT) void k_eval(EvalArgs a) {
    __shared__ double tile[PMAX * PMAX];
    __shared__ double D[PMAX * PMAX], D2[PMAX * PMAX];
    const int cl = blockIdx.x;
    const int li = cl % a.geo.n1, lj = cl / a.geo.n1;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q;
    load_dmat(a.D, D, p * p);
    load_dmat(a.D2, D2, p * p);
    tile_from_canonical(a.geo, li, lj, a.u, tile);
    const int64_t base = (int64_t)cl * q2;
    for (int k = threadIdx.x; k < q2; k += NT) {
        const int64_t gi = base + k;
        const double Lu = tile_L(tile, D, D2, p, q, a.coef, a.geo.n_int, gi, k);
        const double u = tile[(k / q + 1) * p + (k % q) + 1];
        if (a.rhs) {
            // refinement residual of (I - gamma_dt L) u = rhs at interior nodes
            a.r_int[gi] = a.rhs[gi] - (u - a.gamma_dt * Lu);
        } else {
            a.Lu[gi] = Lu;
            const double qv = a.q_src ? a.q_scale * a.q_src[gi] : 0.0;
            a.F[gi] = qv + gpoly(a.g, u);
        }
    }
    if (a.rhs) {
        // coordinate-direction fluxes on the four leaf edges, [leaf][e][m]
        for (int k = threadIdx.x; k < 4 * q; k += NT) {
            const int e = k / q, m = k % q;
            const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * p);
            double f = 0.0;
            if (e < 2) {
                for (int c = 0; c < p; ++c) f = fma(dr[c], tile[(m + 1) * p + c], f);
            } else {
                for (int c = 0; c < p; ++c) f = fma(dr[c], tile[c * p + m + 1], f);
            }
            a.flux[(int64_t)cl * 4 * q + k] = f;
        }
    }
}

// interface residual r3 = jump - (flux_alpha - flux_beta), interface-indexed
__global__ void k_jump(LeafGeo g, const double *flux, const double *jump, double *r3, int64_t n_iface) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_iface) return;
    const int q = g.q;
    const int64_t nv = (int64_t)(g.n1 - 1) * g.n2 * q;
    int ia, ja, ib, jb, ea, eb, m;
    if (t < nv) {
        const int k = (int)(t / ((int64_t)g.n2 * q)) + 1;
        const int rem = (int)(t % ((int64_t)g.n2 * q));
        const int j = rem / q;
        m = rem % q;
        ia = k - 1; ja = j; ea = 1;
        ib = k; jb = j; eb = 0;
    } else {
        const int64_t u = t - nv;
        const int k = (int)(u / ((int64_t)g.n1 * q)) + 1;
        const int rem = (int)(u % ((int64_t)g.n1 * q));
        const int i = rem / q;
        m = rem % q;
        ia = i; ja = k - 1; ea = 3;
        ib = i; jb = k; eb = 2;
    }
    const double fa = flux[((int64_t)ja * g.n1 + ia) * 4 * q + ea * q + m];
    const double fb = flux[((int64_t)jb * g.n1 + ib) * 4 * q + eb * q + m];
    r3[t] = (jump ? jump[t] : 0.0) - (fa - fb);
}

// =======================================================================================
// step completion (interior ARK update, boundary data, interface lines)
// =======================================================================================
struct UpdateArgs {
    int64_t n_int;
    const double *un;
    double *unew;
    const double *Lu, *F;
    double cb[8], cbh[8];
    int s;
};

__global__ void k_update_interior(UpdateArgs a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_int) return;
    double v = a.un[k];
    for (int j = 0; j < a.s; ++j) {
        v += a.cb[j] * a.Lu[j * a.n_int + k];
        v += a.cbh[j] * a.F[j * a.n_int + k];
    }
    a.unew[k] = v;
}

__global__ void k_scatter_boundary(const double *f, const int *bnd_glob, double *u, int64_t nb) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb) u[bnd_glob[k]] = f ? f[k] : 0.0;
}

// Flux continuity along one grid line of leaves: lower e_{k-1} + diag e_k + upper e_{k+1}
// = sum_m D[0][m] u^beta(m) - sum_m D[p-1][m] u^alpha(m), k = 1..n-1, with e_0, e_n the
// boundary values; solved by the Thomas algorithm (diagonally dominant: |diag| >> |lower|+|upper|).
struct LineArgs {
    LeafGeo geo;
    double *u;
    const double *D;          // p*p
    const double *cp;         // Thomas factors: cp[k], k = 1..nmax-1
    const double *inv_den;    // 1 / (diag - lower cp[k-1])
};

__global__ void k_interface_lines(LineArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const LeafGeo &g = a.geo;
    const int q = g.q, p = g.p, q2 = q * q;
    const int nvs = g.n2 * q;   // systems along horizontal rows (vertical-edge unknowns)
    const int nhs = g.n1 * q;
    if (t >= nvs + nhs) return;
    const bool vert = t < nvs;
    const int n = vert ? g.n1 : g.n2;
    if (n < 2) return;
    const int line = vert ? t / q : (t - nvs) / q;   // leaf row j (vert) or column i (horz)
    const int m0 = (vert ? t : t - nvs) % q;          // local node index along the edge
    const double lower = a.D[(p - 1) * p + 0];
    auto unk = [&](int k) -> int64_t {
        return vert ? g.n_int + ((int64_t)k * g.n2 + line) * q + m0
                    : g.n_int + g.n_vert + ((int64_t)k * g.n1 + line) * q + m0;
    };
    auto interior = [&](int leafk, int c) -> double {   // c = 1..q along the line direction
        if (vert) return a.u[((int64_t)line * g.n1 + leafk) * q2 + (int64_t)m0 * q + (c - 1)];
        return a.u[((int64_t)leafk * g.n1 + line) * q2 + (int64_t)(c - 1) * q + m0];
    };
    const double upper = -a.D[0 * p + (p - 1)];
    const double e0 = a.u[unk(0)], en = a.u[unk(n)];
    double dprev = 0.0;
    for (int k = 1; k < n; ++k) {
        double r = 0.0;
        for (int c = 1; c <= q; ++c) {
            r = fma(a.D[c], interior(k, c), r);
            r = fma(-a.D[(p - 1) * p + c], interior(k - 1, c), r);
        }
        if (k == 1) r -= lower * e0;
        if (k == n - 1) r -= upper * en;
        const double d = (r - (k > 1 ? lower * dprev : 0.0)) * a.inv_den[k];
        a.u[unk(k)] = d;
        dprev = d;
    }
    for (int k = n - 2; k >= 1; --k) a.u[unk(k)] -= a.cp[k] * a.u[unk(k + 1)];
}

__global__ void k_zero(double *p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0.0;
}

// =======================================================================================
// build kernels
// =======================================================================================
struct BuildLeafArgs {
    LeafGeo geo;
    const int *leaf_ij;
    const double *coef, *D, *D2;
    double gamma_dt;
};

// A_ii of A = I - gdt L on every leaf (heap order), column-major q2 x q2 (Sec. 2.1, eq. 5)
__global__ __launch_bounds__(NT) void k_leaf_assemble(BuildLeafArgs a, double *W) {
    __shared__ double D[PMAX * PMAX], D2[PMAX * PMAX];
    const int leaf = blockIdx.y;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q;
    load_dmat(a.D, D, p * p);
    load_dmat(a.D2, D2, p * p);
    __syncthreads();
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int64_t n_int = a.geo.n_int;
    const int64_t tot = (int64_t)q2 * q2;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        const int r = (int)(idx % q2), c = (int)(idx / q2);
        const int a1 = r % q + 1, b1 = r / q + 1, a2 = c % q + 1, b2 = c / q + 1;
        const int64_t gi = base + r;
        const double gdt = a.gamma_dt;
        double v = 0.0;
        if (b1 == b2) v += -gdt * a.coef[gi] * D2[a1 * p + a2] - gdt * a.coef[2 * n_int + gi] * D[a1 * p + a2];
        if (a1 == a2) v += -gdt * a.coef[n_int + gi] * D2[b1 * p + b2] - gdt * a.coef[3 * n_int + gi] * D[b1 * p + b2];
        if (r == c) v += 1.0 - gdt * a.coef[4 * n_int + gi];
        W[(int64_t)leaf * tot + idx] = v;
    }
}

// S_leaf = -A_ii^{-1} A_ib (eq. 6); A_ib has q nonzeros per boundary column.
__global__ __launch_bounds__(NT) void k_leaf_S(BuildLeafArgs a, const double *ainv, double *S) {
    __shared__ double D[PMAX * PMAX], D2[PMAX * PMAX];
    const int leaf = blockIdx.y;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q;
    load_dmat(a.D, D, p * p);
    load_dmat(a.D2, D2, p * p);
    __syncthreads();
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int64_t n_int = a.geo.n_int;
    const double gdt = a.gamma_dt;
    const double *Ai = ainv + (int64_t)leaf * q2 * q2;
    const int64_t tot = (int64_t)q2 * nb;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        const int r = (int)(idx % q2), col = (int)(idx / q2);
        const int e = col / q, m = col % q;
        double s = 0.0;
        for (int c = 1; c <= q; ++c) {
            int rho;           // interior row of A_ib touching this boundary node
            double coefv;
            if (e < 2) {       // left / right edge node (a' = 0 or p-1, b = m+1): rows (c, m+1)
                rho = m * q + (c - 1);
                const int ap = (e == 0) ? 0 : p - 1;
                const int64_t gi = base + rho;
                coefv = -gdt * a.coef[gi] * D2[c * p + ap] - gdt * a.coef[2 * n_int + gi] * D[c * p + ap];
            } else {           // bottom / top edge node (a = m+1, b' = 0 or p-1): rows (m+1, c)
                rho = (c - 1) * q + m;
                const int bp = (e == 2) ? 0 : p - 1;
                const int64_t gi = base + rho;
                coefv = -gdt * a.coef[n_int + gi] * D2[c * p + bp] - gdt * a.coef[3 * n_int + gi] * D[c * p + bp];
            }
            s = fma(Ai[(int64_t)rho * q2 + r], coefv, s);
        }
        S[(int64_t)leaf * tot + idx] = -s;
    }
}

// T_leaf = flux rows applied to [S u_b; u_b]: coordinate-direction derivative on each edge
__global__ __launch_bounds__(NT) void k_leaf_T(BuildLeafArgs a, const double *S, double *T) {
    __shared__ double D[PMAX * PMAX];
    const int leaf = blockIdx.y;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q;
    load_dmat(a.D, D, p * p);
    __syncthreads();
    const double *Sl = S + (int64_t)leaf * q2 * nb;
    const int64_t tot = (int64_t)nb * nb;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        const int row = (int)(idx % nb), col = (int)(idx / nb);
        const int e = row / q, m = row % q;
        const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * p);
        double v = 0.0;
        for (int c = 1; c <= q; ++c) {
            const int rho = (e < 2) ? m * q + (c - 1) : (c - 1) * q + m;
            v = fma(dr[c], Sl[(int64_t)col * q2 + rho], v);
        }
        // direct boundary terms: the two edge nodes on the same tile line
        const int lo = (e < 2) ? 0 * q + m : 2 * q + m;    // left or bottom node of the line
        const int hi = (e < 2) ? 1 * q + m : 3 * q + m;    // right or top node of the line
        if (col == lo) v += dr[0];
        if (col == hi) v += dr[p - 1];
        T[(int64_t)leaf * tot + idx] = v;
    }
}

// Gather the merge blocks of level-l nodes from their children's DtN maps (column-major):
// M = T^a_33 - T^b_33, B = [-T^a_31 | T^b_32], Cm = [T^a_13; T^b_23], Tn = diag(T^a_11, T^b_22).
struct MergeArgs {
    int n1, n2, n3, n12, nbc;
    const int *a1, *a3, *b2, *b3;
    const double *Tc;
    double *M, *B, *Cm, *Tn;
};

__global__ __launch_bounds__(NT) void k_merge_gather(MergeArgs a) {
    const int node = blockIdx.y;
    const int64_t nbc2 = (int64_t)a.nbc * a.nbc;
    const double *Ta = a.Tc + (int64_t)(2 * node) * nbc2;
    const double *Tb = a.Tc + (int64_t)(2 * node + 1) * nbc2;
    auto ta = [&](int r, int c) { return Ta[(int64_t)c * a.nbc + r]; };
    auto tb = [&](int r, int c) { return Tb[(int64_t)c * a.nbc + r]; };
    const int n3 = a.n3, n12 = a.n12, n1 = a.n1;
    const int64_t sM = (int64_t)n3 * n3, sB = (int64_t)n3 * n12, sT = (int64_t)n12 * n12;
    const int64_t tot = sM + 2 * sB + (a.Tn ? sT : 0);
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        if (idx < sM) {
            const int r = (int)(idx % n3), c = (int)(idx / n3);
            a.M[node * sM + idx] = ta(a.a3[r], a.a3[c]) - tb(a.b3[r], a.b3[c]);
        } else if (idx < sM + sB) {
            const int64_t k = idx - sM;
            const int r = (int)(k % n3), c = (int)(k / n3);
            a.B[node * sB + k] = (c < n1) ? -ta(a.a3[r], a.a1[c]) : tb(a.b3[r], a.b2[c - n1]);
        } else if (idx < sM + 2 * sB) {
            const int64_t k = idx - sM - sB;
            const int r = (int)(k % n12), c = (int)(k / n12);
            a.Cm[node * sB + k] = (r < n1) ? ta(a.a1[r], a.a3[c]) : tb(a.b2[r - n1], a.b3[c]);
        } else {
            const int64_t k = idx - sM - 2 * sB;
            const int r = (int)(k % n12), c = (int)(k / n12);
            double v = 0.0;
            if (r < n1 && c < n1) v = ta(a.a1[r], a.a1[c]);
            else if (r >= n1 && c >= n1) v = tb(a.b2[r - n1], a.b2[c - n1]);
            a.Tn[node * sT + k] = v;
        }
    }
}

// ---- Gauss-Jordan inversion with partial pivoting, batched, column-major --------------
// Step k picks the unused row with the largest |W[i][k]|, scales it and eliminates column
// k from every other row in place; rows are never swapped.  After n steps with pivot rows
// r_0..r_{n-1}, inv(A)[k][r_j] = W[r_k][j].
__global__ __launch_bounds__(NT) void k_gj_pivot(double *W, int n, int k, unsigned char *used,
                                                 int *order, double *colbuf, double *rowbuf,
                                                 int *sing) {
    __shared__ double bv[NT];
    __shared__ int bi[NT];
    const int b = blockIdx.x;
    double *Wb = W + (int64_t)b * n * n;
    unsigned char *ub = used + (int64_t)b * n;
    double best = -1.0;
    int besti = n;
    for (int i = threadIdx.x; i < n; i += NT) {
        if (!ub[i]) {
            const double v = fabs(Wb[(int64_t)k * n + i]);
            if (v > best || (v == best && i < besti)) {
                best = v;
                besti = i;
            }
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = besti;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const double v2 = bv[threadIdx.x + off];
            const int i2 = bi[threadIdx.x + off];
            if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
                bv[threadIdx.x] = v2;
                bi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    int pr = bi[0];
    double piv = 0.0;
    if (pr < n) piv = Wb[(int64_t)k * n + pr];
    if (pr >= n || piv == 0.0 || !isfinite(piv)) {
        if (threadIdx.x == 0) atomicExch(sing, 1);
        if (pr >= n) pr = 0;
        piv = 1.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ub[pr] = 1;
        order[(int64_t)b * n + k] = pr;
    }
    const double ip = 1.0 / piv;
    for (int i = threadIdx.x; i < n; i += NT) {
        colbuf[(int64_t)b * n + i] = Wb[(int64_t)k * n + i];
        rowbuf[(int64_t)b * n + i] = (i == k) ? ip : Wb[(int64_t)i * n + pr] * ip;
    }
}

__global__ __launch_bounds__(NT) void k_gj_update(double *W, int n, int nb, int k, const int *order,
                                                  const double *colbuf, const double *rowbuf) {
    const int64_t nn = (int64_t)n * n;
    const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (idx >= nn * nb) return;
    const int b = (int)(idx / nn);
    const int64_t rem = idx - b * nn;
    const int j = (int)(rem / n), i = (int)(rem % n);
    const int pr = order[(int64_t)b * n + k];
    const double *cb = colbuf + (int64_t)b * n;
    const double *rb = rowbuf + (int64_t)b * n;
    if (i == pr) W[idx] = rb[j];
    else if (j == k) W[idx] = -cb[i] * rb[k];
    else W[idx] = fma(-cb[i], rb[j], W[idx]);
}

__global__ void k_gj_unpermute(const double *W, double *out, int n, int nb, const int *order) {
    const int64_t nn = (int64_t)n * n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nn * nb) return;
    const int b = (int)(idx / nn);
    const int64_t rem = idx - b * nn;
    const int j = (int)(rem / n), k = (int)(rem % n);
    const int *o = order + (int64_t)b * n;
    // out[k][o[j]] = W[o[k]][j]  (column-major)
    out[b * nn + (int64_t)o[j] * n + k] = W[b * nn + (int64_t)j * n + o[k]];
}

// ---- batched FP64 GEMM on the matrix cores ----------------------------------------------
// C = alpha A B + beta C, column-major, 64x64 tile per workgroup, each wave a 32x32
// sub-tile of 2x2 v_mfma_f64_16x16x4 blocks; K staged through LDS 16 at a time.
typedef double dvec4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
    int M, N, K;
    const double *A; int lda; int64_t sA;
    const double *B; int ldb; int64_t sB;
    double *C; int ldc; int64_t sC;
    double alpha, beta;
};

__global__ __launch_bounds__(NT) void k_dgemm(GemmArgs g) {
    constexpr int TM = 64, TN = 64, TK = 16;
    __shared__ double As[TK][TM + 1];
    __shared__ double Bs[TK][TN + 1];
    const int bz = blockIdx.z;
    const double *A = g.A + bz * g.sA;
    const double *B = g.B + bz * g.sB;
    double *C = g.C + bz * g.sC;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    dvec4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = dvec4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < g.K; k0 += TK) {
        for (int e = t; e < TM * TK; e += NT) {
            const int i = e % TM, kk = e / TM;
            const int gm = m0 + i, gk = k0 + kk;
            As[kk][i] = (gm < g.M && gk < g.K) ? A[(int64_t)gk * g.lda + gm] : 0.0;
        }
        for (int e = t; e < TN * TK; e += NT) {
            const int kk = e % TK, j = e / TK;
            const int gn = n0 + j, gk = k0 + kk;
            Bs[kk][j] = (gn < g.N && gk < g.K) ? B[(int64_t)gn * g.ldb + gk] : 0.0;
        }
        __syncthreads();
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = As[kk + lk][wm * 32 + x * 16 + li];
#pragma unroll
            for (int y = 0; y < 2; ++y) bv[y] = Bs[kk + lk][wn * 32 + y * 16 + li];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
        }
        __syncthreads();
    }
    // v_mfma_f64_16x16x4: lane l, register r holds D[l/16 + 4r][l%16]
    const int cj = lane & 15, ci = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + x * 16 + ci + 4 * r;
                const int col = n0 + wn * 32 + y * 16 + cj;
                if (row < g.M && col < g.N) {
                    double *c = C + (int64_t)col * g.ldc + row;
                    const double v = g.alpha * acc[x][y][r];
                    *c = (g.beta == 0.0) ? v : fma(g.beta, *c, v);
                }
            }
}

// ---- pack a column-major operator into the streaming layout ------------------------------
struct PackArgs {
    int R, C, vw, rp, G, S, ntile, kch;
    int64_t tile_elems, node_elems, total;
    const double *src0; int ld0; int64_t stride0; int rows0;
    const double *src1; int ld1; int64_t stride1;
    void *dst;
};

template <typename T>
__global__ void k_pack(PackArgs a) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.total) return;
    const int64_t node = idx / a.node_elems;
    int64_t rem = idx - node * a.node_elems;
    const int64_t blk = rem / a.tile_elems;
    rem -= blk * a.tile_elems;
    const int tile = (int)(blk / a.kch), chunk = (int)(blk % a.kch);
    const int act = a.rp * a.G;
    const int s = (int)(rem / ((int64_t)act * a.vw));
    const int tv = (int)(rem % ((int64_t)act * a.vw));
    const int t = tv / a.vw, v = tv % a.vw;
    const int g = t / a.rp, r = t % a.rp;
    const int row = tile * a.rp * a.vw + r * a.vw + v;
    const int col = chunk * a.S * a.G + s * a.G + g;
    double val = 0.0;
    if (row < a.R && col < a.C) {
        if (row < a.rows0) val = a.src0[node * a.stride0 + (int64_t)col * a.ld0 + row];
        else val = a.src1[node * a.stride1 + (int64_t)col * a.ld1 + (row - a.rows0)];
    }
    reinterpret_cast<T *>(a.dst)[idx] = (T)val;
}

// =======================================================================================
// launchers
// =======================================================================================
static LeafGeo geo_of(const hps_op *op) {
    return LeafGeo{op->grid.n1, op->grid.n2, op->q, op->p, op->n_int, op->n_vert};
}

static inline unsigned nblk(int64_t n, int t = NT) { return (unsigned)((n + t - 1) / t); }

// ---- profiling ---------------------------------------------------------------------------
const char *const kKernelFamilyNames[KF_COUNT] = {
    "leaf_up_fp64", "leaf_up_fp32", "level_up_fp64", "level_up_fp32", "level_down_fp64",
    "level_down_fp32", "leaf_down_fp64", "leaf_down_fp32", "eval", "residual", "update"};

hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

Profiler::~Profiler() {
    for (auto &r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(Profiler *p_, int fam_, hipStream_t st_) : p(p_), fam(fam_), st(st_) {
    if (p && p->on) {
        a = p->get();
        if (a) (void)hipEventRecord(a, st);
    }
}

ProfScope::~ProfScope() {
    if (p && p->on && a) {
        hipEvent_t b = p->get();
        if (b) {
            (void)hipEventRecord(b, st);
            p->recs.push_back(Profiler::Rec{fam, a, b});
        }
    }
}

int launch_leaf_up(const hps_op *op, bool fp32, const double *body, const double *un,
                   const double *Lu, const double *F, const StageCoefs *sc, double *rhs_copy,
                   hipStream_t st) {
    ProfScope ps_(&op->prof, fp32 ? KF_LEAF_UP32 : KF_LEAF_UP64, st);
    LeafUpArgs a{};
    a.ainv = view(fp32 ? op->ainv32 : op->ainv64);
    a.leaf_ij = op->leaf_ij;
    a.geo = geo_of(op);
    a.body = body;
    a.un = un;
    a.Lu = Lu;
    a.F = F;
    if (sc) a.sc = *sc;
    a.rhs_copy = rhs_copy;
    a.D = op->D;
    a.w_out = op->w_leaf;
    a.h_out = op->h_leaf;
    if (fp32) hipLaunchKernelGGL(k_leaf_up<float>, dim3(op->nleaves), dim3(NT), 0, st, a);
    else hipLaunchKernelGGL(k_leaf_up<double>, dim3(op->nleaves), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

static LevelArgs level_args(const hps_op *op, int l, bool fp32, bool up) {
    const Level &L = op->lv[l];
    LevelArgs a{};
    a.pn = view(up ? (fp32 ? L.xu32 : L.xu64) : (fp32 ? L.s32 : L.s64));
    a.n1 = L.n1; a.n2 = L.n2; a.n3 = L.n3; a.n12 = L.n12; a.nbc = L.nbc;
    a.a1 = L.a1; a.a3 = L.a3; a.b2 = L.b2; a.b3 = L.b3;
    a.j3i = L.j3i;
    const bool child_leaf = (l == op->L - 1);
    a.hc = child_leaf ? op->h_leaf : op->lv[l + 1].h;
    a.w3 = L.w3;
    a.h = L.h;
    a.ub = L.ub;
    a.ubc = child_leaf ? op->ub_leaf : op->lv[l + 1].ub;
    a.root_map = op->root_map;
    a.root = (l == 0);
    a.part = L.part;
    return a;
}

int launch_levels_up(const hps_op *op, bool fp32, const double *jump, hipStream_t st) {
    ProfScope ps_(&op->prof, fp32 ? KF_LEVEL_UP32 : KF_LEVEL_UP64, st);
    for (int l = op->L - 1; l >= 0; --l) {
        LevelArgs a = level_args(op, l, fp32, true);
        a.r3 = jump;
        const unsigned nb = (unsigned)(op->lv[l].nodes * a.pn.ntile * a.pn.kch);
        if (fp32) hipLaunchKernelGGL((k_level<float, true>), dim3(nb), dim3(NT), 0, st, a);
        else hipLaunchKernelGGL((k_level<double, true>), dim3(nb), dim3(NT), 0, st, a);
        HPS_LAUNCHED();
        if (a.pn.kch > 1) {
            hipLaunchKernelGGL(k_level_finalize<true>, dim3(op->lv[l].nodes * a.pn.ntile), dim3(NT),
                               0, st, a, fp32 ? 4 : 2);
            HPS_LAUNCHED();
        }
    }
    return HPS_OK;
}

// single-leaf tree: the leaf boundary is the domain boundary
__global__ void k_root_leaf_ub(const double *dir, const int *root_map, double *ub, int nb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nb) ub[t] = dir ? dir[root_map[t]] : 0.0;
}

int launch_levels_down(const hps_op *op, bool fp32, const double *dirichlet, hipStream_t st) {
    ProfScope ps_(&op->prof, fp32 ? KF_LEVEL_DOWN32 : KF_LEVEL_DOWN64, st);
    if (op->L == 0) {
        hipLaunchKernelGGL(k_root_leaf_ub, dim3(1), dim3(NT), 0, st, dirichlet, (const int *)op->root_map,
                           op->ub_leaf, 4 * op->q);
        HPS_LAUNCHED();
        return HPS_OK;
    }
    for (int l = 0; l < op->L; ++l) {
        LevelArgs a = level_args(op, l, fp32, false);
        a.dir = dirichlet;
        const unsigned nb = (unsigned)(op->lv[l].nodes * a.pn.ntile * a.pn.kch);
        if (fp32) hipLaunchKernelGGL((k_level<float, false>), dim3(nb), dim3(NT), 0, st, a);
        else hipLaunchKernelGGL((k_level<double, false>), dim3(nb), dim3(NT), 0, st, a);
        HPS_LAUNCHED();
        if (a.pn.kch > 1) {
            hipLaunchKernelGGL(k_level_finalize<false>, dim3(op->lv[l].nodes * a.pn.ntile), dim3(NT),
                               0, st, a, fp32 ? 4 : 2);
            HPS_LAUNCHED();
        }
    }
    return HPS_OK;
}

int launch_leaf_down(const hps_op *op, bool fp32, int mode, double *u, double *Lu, double *F,
                     const double *q_src, double q_scale, GPoly g, hipStream_t st) {
    ProfScope ps_(&op->prof, fp32 ? KF_LEAF_DOWN32 : KF_LEAF_DOWN64, st);
    LeafDownArgs a{};
    a.sl = view(fp32 ? op->sleaf32 : op->sleaf64);
    a.leaf_ij = op->leaf_ij;
    a.geo = geo_of(op);
    a.ub = op->ub_leaf;
    a.w = op->w_leaf;
    a.D = op->D;
    a.D2 = op->D2;
    a.coef = op->coef;
    a.mode = mode;
    a.u = u;
    a.Lu = Lu;
    a.F = F;
    a.q_src = q_src;
    a.q_scale = q_scale;
    a.g = g;
    a.norms = reinterpret_cast<unsigned long long *>(op->ir_norms);
    if (fp32) hipLaunchKernelGGL(k_leaf_down<float>, dim3(op->nleaves), dim3(NT), 0, st, a);
    else hipLaunchKernelGGL(k_leaf_down<double>, dim3(op->nleaves), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_eval(const hps_op *op, const double *u, double *Lu, double *F, const double *q_src,
                double q_scale, GPoly g, hipStream_t st) {
    ProfScope ps_(&op->prof, KF_EVAL, st);
    EvalArgs a{};
    a.geo = geo_of(op);
    a.u = u;
    a.D = op->D;
    a.D2 = op->D2;
    a.coef = op->coef;
    a.Lu = Lu;
    a.F = F;
    a.q_src = q_src;
    a.q_scale = q_scale;
    a.g = g;
    hipLaunchKernelGGL(k_eval, dim3(op->nleaves), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_residual(const hps_op *op, const double *u, const double *rhs, const double *jump,
                    double *r_int, double *r3, hipStream_t st) {
    ProfScope ps_(&op->prof, KF_RESIDUAL, st);
    EvalArgs a{};
    a.geo = geo_of(op);
    a.u = u;
    a.D = op->D;
    a.D2 = op->D2;
    a.coef = op->coef;
    a.rhs = rhs;
    a.gamma_dt = op->gamma_dt;
    a.r_int = r_int;
    a.flux = op->ir_flux;
    hipLaunchKernelGGL(k_eval, dim3(op->nleaves), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    if (op->n_iface > 0) {
        hipLaunchKernelGGL(k_jump, dim3(nblk(op->n_iface)), dim3(NT), 0, st, geo_of(op),
                           (const double *)op->ir_flux, jump, r3, op->n_iface);
        HPS_LAUNCHED();
    }
    return HPS_OK;
}

int launch_update(const hps_op *op, const double *un, double *unew, const double *Lu,
                  const double *F, const double *cb, const double *cbh, int s,
                  const double *f_end, hipStream_t st) {
    ProfScope ps_(&op->prof, KF_UPDATE, st);
    UpdateArgs a{};
    a.n_int = op->n_int;
    a.un = un;
    a.unew = unew;
    a.Lu = Lu;
    a.F = F;
    a.s = s;
    for (int j = 0; j < s; ++j) {
        a.cb[j] = cb[j];
        a.cbh[j] = cbh[j];
    }
    hipLaunchKernelGGL(k_update_interior, dim3(nblk(op->n_int)), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    int rc = launch_scatter_boundary(op, f_end, unew, st);
    if (rc) return rc;
    LineArgs la{};
    la.geo = geo_of(op);
    la.u = unew;
    la.D = op->D;
    la.cp = op->tri_cp;
    la.inv_den = op->tri_cp + op->tri_stride;
    const int nsys = op->grid.n2 * op->q + op->grid.n1 * op->q;
    hipLaunchKernelGGL(k_interface_lines, dim3(nblk(nsys, 64)), dim3(64), 0, st, la);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_scatter_boundary(const hps_op *op, const double *f, double *u, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_boundary, dim3(nblk(op->n_bdry)), dim3(NT), 0, st, f,
                       (const int *)op->bnd_glob, u, op->n_bdry);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_zero(double *p, int64_t n, hipStream_t st) {
    if (n <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(NT), 0, st, p, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

static BuildLeafArgs build_leaf_args(const hps_op *op) {
    return BuildLeafArgs{geo_of(op), op->leaf_ij, op->coef, op->D, op->D2, op->gamma_dt};
}

int launch_leaf_assemble(const hps_op *op, double *W, hipStream_t st) {
    const int64_t tot = (int64_t)op->q2 * op->q2;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 64);
    hipLaunchKernelGGL(k_leaf_assemble, dim3(bx, op->nleaves), dim3(NT), 0, st, build_leaf_args(op), W);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_leaf_S(const hps_op *op, const double *ainv, double *S, hipStream_t st) {
    const int64_t tot = (int64_t)op->q2 * 4 * op->q;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 64);
    hipLaunchKernelGGL(k_leaf_S, dim3(bx, op->nleaves), dim3(NT), 0, st, build_leaf_args(op), ainv, S);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_leaf_T(const hps_op *op, const double *S, double *T, hipStream_t st) {
    const int64_t tot = (int64_t)16 * op->q * op->q;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 64);
    hipLaunchKernelGGL(k_leaf_T, dim3(bx, op->nleaves), dim3(NT), 0, st, build_leaf_args(op), S, T);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_merge_gather(const Level &L, bool root, const double *Tc, double *M, double *B,
                        double *Cm, double *Tn, hipStream_t st) {
    MergeArgs a{L.n1, L.n2, L.n3, L.n12, L.nbc, L.a1, L.a3, L.b2, L.b3, Tc, M, B, Cm, root ? nullptr : Tn};
    const int64_t tot = (int64_t)L.n3 * L.n3 + 2 * (int64_t)L.n3 * L.n12 +
                        (root ? 0 : (int64_t)L.n12 * L.n12);
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 4096);
    hipLaunchKernelGGL(k_merge_gather, dim3(bx, L.nodes), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

int gj_invert(double *W, double *out, int n, int nb, unsigned char *used, int *order,
              double *colbuf, double *rowbuf, int *sing, hipStream_t st) {
    HPS_HIP(hipMemsetAsync(used, 0, (size_t)n * nb, st));
    const int64_t tot = (int64_t)n * n * nb;
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(nb), dim3(NT), 0, st, W, n, k, used, order, colbuf, rowbuf, sing);
        HPS_LAUNCHED();
        hipLaunchKernelGGL(k_gj_update, dim3(nblk(tot)), dim3(NT), 0, st, W, n, nb, k,
                           (const int *)order, (const double *)colbuf, (const double *)rowbuf);
        HPS_LAUNCHED();
    }
    hipLaunchKernelGGL(k_gj_unpermute, dim3(nblk(tot)), dim3(NT), 0, st, (const double *)W, out, n, nb,
                       (const int *)order);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_dgemm(int M, int N, int K, const double *A, int lda, int64_t sA, const double *B,
                 int ldb, int64_t sB, double *C, int ldc, int64_t sC, int batch, double alpha,
                 double beta, hipStream_t st) {
    if (M <= 0 || N <= 0 || batch <= 0) return HPS_OK;
    GemmArgs g{M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta};
    hipLaunchKernelGGL(k_dgemm, dim3(nblk(M, 64), nblk(N, 64), batch), dim3(NT), 0, st, g);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_pack(const Panel &pn, const double *src0, int ld0, int64_t stride0, int rows0,
                const double *src1, int ld1, int64_t stride1, hipStream_t st) {
    PackArgs a{};
    a.R = pn.R; a.C = pn.C; a.vw = pn.vw; a.rp = pn.rp; a.G = pn.G; a.S = pn.S;
    a.ntile = pn.ntile; a.kch = pn.kch;
    a.tile_elems = pn.tile_elems; a.node_elems = pn.node_elems;
    a.total = pn.node_elems * pn.nodes;
    a.src0 = src0; a.ld0 = ld0; a.stride0 = stride0; a.rows0 = rows0;
    a.src1 = src1; a.ld1 = ld1; a.stride1 = stride1;
    a.dst = pn.data;
    if (pn.vw == 2) hipLaunchKernelGGL(k_pack<double>, dim3(nblk(a.total)), dim3(NT), 0, st, a);
    else hipLaunchKernelGGL(k_pack<float>, dim3(nblk(a.total)), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

}  // namespace hps
