// HIP kernels of the RKHPS per-stage solve on gfx950.
//
// Method: Chen, Appelo, Babb & Martinsson, arXiv 2306.02526.
//   Sec. 2.1 eqs. (5)-(6): leaf solution operator S = -A_ii^{-1} A_ib and DtN map T;
//   the merge formulas after eqs. (7)-(8); Algorithm 1 (solve stage) extended by the
//   particular-solution (body load) and interface-jump terms; Sec. 3.1 eqs. (9)-(11):
//   stage right-hand sides, stage boundary data and the step update.
//
// Every solve kernel streams a packed operator (struct Panel) from HBM exactly once: the
// storage order equals the order in which the workgroup's lanes read it, so each loop
// iteration of a workgroup is one contiguous run of 16-byte loads.  The first loads are
// issued before the workgroup gathers its input vector, which hides the gather latency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "hps_device.h"

namespace hps {

constexpr int PF = 16;   // operator loads issued before the input gather (level panels keep S <= 16,
                         // so a workgroup's whole operator block is in flight during the gather)
constexpr int UNR = 8;   // operator loads in flight in the streaming loop
// Level panels with at most PF_SMALL columns per lane (the bottom levels: many small nodes,
// more workgroups than stay resident at the full kernel's register use) take a variant with
// fewer load registers, so that 8 waves per SIMD fit and the grid runs in one round.
constexpr int PF_SMALL = 4;

__device__ __forceinline__ double gpoly(const GPoly &g, double u) {
    if (g.kind == 0) return 0.0;
    return g.g0 + u * (g.g1 + u * (g.g2 + u * g.g3));
}

// Sum of the nsl slice partials red[s * rows + r] for row r = threadIdx.x < rows, in a fixed
// order.  Many slices (thin row tiles) are first added in groups of 8 in parallel (into
// red2), so no thread runs a long dependent chain of LDS reads.  Every thread calls it.
__device__ __forceinline__ double slice_sum(const double *red, double *red2, int nsl, int rows) {
    const int t = threadIdx.x;
    double y = 0.0;
    if (nsl <= 16) {
        if (t < rows)
            for (int s2 = 0; s2 < nsl; ++s2) y += red[s2 * rows + t];
        return y;
    }
    const int ng = (nsl + 7) / 8;   // ng * rows <= NT / 8 + rows
    if (t < ng * rows) {
        const int g = t / rows, r = t % rows;
        const int s1 = min(nsl, g * 8 + 8);
        double z = 0.0;
        for (int s2 = g * 8; s2 < s1; ++s2) z += red[s2 * rows + r];
        red2[g * rows + r] = z;
    }
    __syncthreads();
    if (t < rows)
        for (int g = 0; g < ng; ++g) y += red2[g * rows + t];
    return y;
}

// slice_sum for NC right-hand sides at once: component c's slices at red + c * rstride,
// its group sums at red2 + c * 64.  The same additions in the same order as slice_sum, for
// every component, with the barriers shared.  Every thread calls it; y[c] is valid in
// threads t < rows.
template <int NC>
__device__ __forceinline__ void slice_sum_n(const double *red, int rstride, double *red2, int nsl, int rows,
                                            double y[NC]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c] = 0.0;
    if (nsl <= 16) {
        if (t < rows)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                for (int s2 = 0; s2 < nsl; ++s2) y[c] += red[c * rstride + s2 * rows + t];
        return;
    }
    const int ng = (nsl + 7) / 8;   // ng * rows <= NT / 8 + rows <= 64
    if (t < ng * rows) {
        const int g = t / rows, r = t % rows;
        const int s1 = min(nsl, g * 8 + 8);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double z = 0.0;
            for (int s2 = g * 8; s2 < s1; ++s2) z += red[c * rstride + s2 * rows + r];
            red2[c * 64 + g * rows + r] = z;
        }
    }
    __syncthreads();
    if (t < rows)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            for (int g = 0; g < ng; ++g) y[c] += red2[c * 64 + g * rows + t];
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
    int *cnt;              // split-K arrival counters [nodes][ntile], zero between launches
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

__device__ __forceinline__ double down_input(const LevelArgs &a, const double *dir, int node, int k) {
    if (a.root) return dir ? dir[a.root_map[k]] : 0.0;
    return a.ub[(int64_t)node * a.n12 + k];
}


// One (node, row tile, column chunk) of a level product: workgroup-local index blk.
template <typename T, bool UP, int PFX = PF, int UNRX = UNR>
__device__ __forceinline__ void level_body(const LevelArgs &a, int blk, unsigned char *smem, double *red,
                                           int *s_last) {
    constexpr int VW = 16 / sizeof(T);
    const int kch = a.pn.kch, ntile = a.pn.ntile;
    const int chunk = blk % kch;
    const int tile = (blk / kch) % ntile;
    const int node = blk / (kch * ntile);
    const int SG = a.pn.S * a.pn.G;
    Carve cv{smem};
    T *xs = cv.take<T>(SG);
    T *part = cv.take<T>((size_t)a.pn.G * a.pn.rp * VW);
    PanelStream<T, PFX, UNRX> ps;
    ps.start(reinterpret_cast<const T *>(a.pn.data) + (int64_t)node * a.pn.node_elems +
                 (int64_t)(tile * kch + chunk) * a.pn.tile_elems,
             a.pn.rp, a.pn.G, a.pn.S);
    // operands of the finalisation, loaded now so the tail has no dependent global loads
    // (level tiles have at most NT rows, one per thread)
    const int rows = a.pn.rp * VW;
    const int myrow = tile * rows + threadIdx.x;
    double fin = 0.0;
    int64_t ia = -1, ib = -1;
    if (kch == 1 && (int)threadIdx.x < rows) {
        if (UP) {
            if (!a.root && myrow >= a.n3 && myrow < a.n3 + a.n12) {
                const int m = myrow - a.n3;
                fin = (m < a.n1) ? a.hc[(int64_t)(2 * node) * a.nbc + a.a1[m]]
                                 : a.hc[(int64_t)(2 * node + 1) * a.nbc + a.b2[m - a.n1]];
            }
        } else if (myrow < a.n3) {
            fin = a.w3[(int64_t)node * a.n3 + myrow];
            ia = (int64_t)(2 * node) * a.nbc + a.a3[myrow];
            ib = (int64_t)(2 * node + 1) * a.nbc + a.b3[myrow];
        }
    }
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
                x = down_input(a, a.dir, node, kg);
            }
        }
        xs[k] = (T)x;
    }
    if (!UP) {
        // the J1 / J2 parts of the children's boundary data are the parent's own; the
        // workgroups of the node copy one slice each
        const int nblk_node = ntile * kch, me = tile * kch + chunk;
        const int per = (a.n12 + nblk_node - 1) / nblk_node;
        const int m1 = min(a.n12, (me + 1) * per);
        for (int m = me * per + threadIdx.x; m < m1; m += NT) {
            const double v = down_input(a, a.dir, node, m);
            if (m < a.n1) a.ubc[(int64_t)(2 * node) * a.nbc + a.a1[m]] = v;
            else a.ubc[(int64_t)(2 * node + 1) * a.nbc + a.b2[m - a.n1]] = v;
        }
    }
    __syncthreads();
    ps.finish(xs, part);
    __syncthreads();
    if (kch == 1) {
        // rows x G partial sums: each row is summed over the column groups by several
        // threads, then the slices are added in a fixed order
        const int G = a.pn.G;
        const int nsl = min(G, NT / rows);
        const int t = threadIdx.x;
        const int row = t % rows, sl = t / rows;
        if (sl < nsl) {
            T y = T(0);
            for (int gg = sl; gg < G; gg += nsl) y += part[gg * rows + row];
            red[sl * rows + row] = (double)y;
        }
        __syncthreads();
        const double y = slice_sum(red, red + NT, nsl, rows);
        if (t < rows) {
            if (UP) {
                if (myrow < a.n3) a.w3[(int64_t)node * a.n3 + myrow] = y;
                else if (!a.root && myrow < a.n3 + a.n12) a.h[(int64_t)node * a.n12 + myrow - a.n3] = fin + y;
            } else if (myrow < a.n3) {
                const double u3 = y + fin;
                a.ubc[ia] = u3;
                a.ubc[ib] = u3;
            }
        }
        return;
    }
    // split-K: publish this chunk's partial sums; the last workgroup of the (node, tile)
    // to arrive adds all chunks in a fixed order and finalises (deterministic).
    double *pp = a.part + ((int64_t)node * ntile + tile) * kch * rows;
    for (int idx = threadIdx.x; idx < rows; idx += NT)
        pp[(int64_t)chunk * rows + idx] = panel_sum<T>(part, a.pn.rp, a.pn.G, idx);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *s_last = (atomicAdd(&a.cnt[node * ntile + tile], 1) == kch - 1);
    __syncthreads();
    if (!*s_last) return;
    __threadfence();
    for (int r0 = 0; r0 < rows; r0 += NT) {
        const int nr = min(NT, rows - r0);
        const int nsl = NT / nr;
        const int t = threadIdx.x;
        const int row = t % nr, sl = t / nr;
        if (sl < nsl) {
            double y = 0.0;
            for (int c = sl; c < kch; c += nsl) y += pp[(int64_t)c * rows + r0 + row];
            red[sl * nr + row] = y;
        }
        __syncthreads();
        if (t < nr) {
            double y = 0.0;
            for (int s2 = 0; s2 < nsl; ++s2) y += red[s2 * nr + t];
            if (UP) up_finalize(a, node, tile * rows + r0 + t, y);
            else down_finalize(a, node, tile * rows + r0 + t, y);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.cnt[node * ntile + tile] = 0;
}

template <typename T, bool UP>
__global__ __launch_bounds__(NT) void k_level(LevelArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    __shared__ int s_last;
    level_body<T, UP>(a, blockIdx.x, smem, red, &s_last);
}

// Panels with S <= PF_SMALL: the same product with fewer registers (8 waves per SIMD).
template <typename T, bool UP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_level_small(LevelArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    __shared__ int s_last;
    level_body<T, UP, PF_SMALL, PF_SMALL>(a, blockIdx.x, smem, red, &s_last);
}

template <typename T, bool UP>
static void launch_level(const LevelArgs &a, unsigned nb, size_t lds, hipStream_t st) {
    if (a.pn.S <= PF_SMALL) hipLaunchKernelGGL((k_level_small<T, UP>), dim3(nb), dim3(NT), lds, st, a);
    else hipLaunchKernelGGL((k_level<T, UP>), dim3(nb), dim3(NT), lds, st, a);
}

// One level product of several operators in one launch: workgroup w belongs to entry e,
// base[e] <= w < base[e + 1].
template <typename T, bool UP>
__global__ __launch_bounds__(NT) void k_level_group(const LevelArgs *args, const int *base, int n) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    __shared__ int s_last;
    const int w = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    level_body<T, UP>(args[lo], w - base[lo], smem, red, &s_last);
}

// =======================================================================================
// composed level pairs: two adjacent tree levels swept by one launch per direction
// =======================================================================================
// The products of two adjacent levels are linear maps, so their composition is one matrix
// per node of the upper level (built once, hps_compose.hip).  Upward it takes the
// interface differences d of both children and of the node to both levels' w3 and the
// node's particular fluxes h; downward it takes the node's boundary values and w3 to the
// shared-edge values of the node and of both children.  The top pair (the root and its
// children) is one kernel from the Dirichlet data and the differences below it to the
// shared-edge values of both levels.  Every input and output position comes from a table
// built on the host from the two levels' index maps, relative to the node's four
// grandchildren (whose boundary vectors are contiguous).
enum { PAIR_UP = 0, PAIR_DOWN = 1, PAIR_TOP = 2 };

struct PairArgs {
    PanelView pn;
    int R, C;                    // rows and input columns of the composite operator
    int n3t, n12t, n3c, nbcc;    // |J3|, |J12| of the upper level; |J3| of the lower; grandchild boundary length
    const int *tab;              // the pair's tables
    int t_plus, t_minus, t_j3, t_fin, t_copy;   // their offsets in tab
    const double *hg;            // grandchildren's particular fluxes [4 per node][nbcc]
    const double *r3;            // interface jumps or null
    const int *j3i_t, *j3i_c;    // J3 interface indices of the upper and lower level
    double *h_t, *w3_t, *w3_c;   // upward outputs (downward: w3 is read)
    const double *ub_t;          // the upper level's boundary values [nodes][n12t]
    double *ubg;                 // grandchildren's boundary values [4 per node][nbcc]
    const double *dir;           // top: Dirichlet data (boundary-indexed) or null
    const int *root_map;         // top: root boundary position -> boundary index
};

// input column k of the upward / top gathers: a difference of two grandchild fluxes plus
// the interface jump of the J3 node the column belongs to
__device__ __forceinline__ double pair_diff(const PairArgs &a, int node, int64_t gbase, int k) {
    const int *t = a.tab;
    double x = a.hg[gbase + t[a.t_plus + k]] - a.hg[gbase + t[a.t_minus + k]];
    if (a.r3) {
        const int jc = t[a.t_j3 + k];
        x += jc >= 0 ? a.r3[a.j3i_c[(int64_t)node * 2 * a.n3c + jc]] : a.r3[a.j3i_t[(int64_t)node * a.n3t - jc - 1]];
    }
    return x;
}

template <typename T, int MODE>
__device__ __forceinline__ void pair_body(const PairArgs &a, int blk, unsigned char *smem, double *red) {
    constexpr int VW = 16 / sizeof(T);
    const int ntile = a.pn.ntile;
    const int tile = blk % ntile;
    const int node = blk / ntile;
    const int SG = a.pn.S * a.pn.G;
    Carve cv{smem};
    T *xs = cv.take<T>(SG);
    T *part = cv.take<T>((size_t)a.pn.G * a.pn.rp * VW);
    // without Dirichlet data the top pair's first n12t input columns are zero: the column
    // steps s < n12t / G hold only those columns and are not streamed (their products are
    // zeros, so the sums are the same)
    const int s0 = (MODE == PAIR_TOP && !a.dir) ? a.n12t / a.pn.G : 0;
    PanelStream<T, PF, UNR> ps;
    ps.start(reinterpret_cast<const T *>(a.pn.data) + (int64_t)node * a.pn.node_elems + (int64_t)tile * a.pn.tile_elems +
                 (int64_t)s0 * a.pn.rp * a.pn.G * VW,
             a.pn.rp, a.pn.G, a.pn.S - s0);
    const int rows = a.pn.rp * VW;   // at most NT: one row per thread
    const int myrow = tile * rows + threadIdx.x;
    const int64_t gbase = (int64_t)node * 4 * a.nbcc;
    const int *tab = a.tab;
    // operands of the finalisation, loaded before the stream is consumed
    int kind = -1, idx = 0, p1 = -1, p2 = -1;
    double base = 0.0;
    if ((int)threadIdx.x < rows && myrow < a.R) {
        if (MODE == PAIR_UP) {
            kind = tab[a.t_fin + 3 * myrow];
            idx = tab[a.t_fin + 3 * myrow + 1];
            if (kind == 2) base = a.hg[gbase + tab[a.t_fin + 3 * myrow + 2]];
        } else {
            kind = tab[a.t_fin + 4 * myrow];
            idx = tab[a.t_fin + 4 * myrow + 1];
            p1 = tab[a.t_fin + 4 * myrow + 2];
            p2 = tab[a.t_fin + 4 * myrow + 3];
            if (kind == 1) base = a.w3_t[(int64_t)node * a.n3t + idx];
            else if (kind == 0) base = a.w3_c[(int64_t)node * 2 * a.n3c + idx];
        }
    }
    for (int k = threadIdx.x; k < SG; k += NT) {
        double x = 0.0;
        if (k < a.C) {
            if (MODE == PAIR_UP) {
                x = pair_diff(a, node, gbase, k);
            } else if (MODE == PAIR_DOWN) {
                x = k < a.n12t ? a.ub_t[(int64_t)node * a.n12t + k] : a.w3_t[(int64_t)node * a.n3t + k - a.n12t];
            } else {
                x = k < a.n12t ? (a.dir ? a.dir[a.root_map[k]] : 0.0) : pair_diff(a, 0, 0, k);
            }
        }
        xs[k] = (T)x;
    }
    if (MODE != PAIR_UP) {
        // the node's own boundary values go to the grandchildren unchanged; the node's row
        // tiles copy one slice each
        const int per = (a.n12t + ntile - 1) / ntile;
        const int m1 = min(a.n12t, (tile + 1) * per);
        for (int m = tile * per + threadIdx.x; m < m1; m += NT) {
            const double v = MODE == PAIR_DOWN ? a.ub_t[(int64_t)node * a.n12t + m]
                                               : (a.dir ? a.dir[a.root_map[m]] : 0.0);
            a.ubg[gbase + tab[a.t_copy + m]] = v;
        }
    }
    __syncthreads();
    ps.finish(xs + s0 * a.pn.G, part);
    __syncthreads();
    const int G = a.pn.G;
    const int nsl = min(G, NT / rows);
    const int t = threadIdx.x;
    const int row = t % rows, sl = t / rows;
    if (sl < nsl) {
        T y = T(0);
        for (int gg = sl; gg < G; gg += nsl) y += part[gg * rows + row];
        red[sl * rows + row] = (double)y;
    }
    __syncthreads();
    const double y = slice_sum(red, red + NT, nsl, rows);
    if (t < rows && myrow < a.R) {
        if (MODE == PAIR_UP) {
            if (kind == 0) a.w3_c[(int64_t)node * 2 * a.n3c + idx] = y;
            else if (kind == 1) a.w3_t[(int64_t)node * a.n3t + idx] = y;
            else a.h_t[(int64_t)node * a.n12t + idx] = base + y;
        } else {
            const double u3 = y + base;
            a.ubg[gbase + p1] = u3;
            if (p2 >= 0) a.ubg[gbase + p2] = u3;
        }
    }
}

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_pair(PairArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    pair_body<T, MODE>(a, blockIdx.x, smem, red);
}

// A composite product for NC right-hand sides (component c's buffers in A.c[c]; the panel
// and tables of A.c[0]): the operator block is streamed once for all of them, and every
// component's arithmetic is pair_body's, in the same order.
template <int NC>
struct PairArgsN {
    PairArgs c[NC];
};

template <int NC, int MODE>
__device__ __forceinline__ void pair_sys_body(const PairArgsN<NC> &A, int blk, unsigned char *smem) {
    constexpr int VW = 2;
    const PairArgs &a = A.c[0];
    const int ntile = a.pn.ntile;
    const int tile = blk % ntile;
    const int node = blk / ntile;
    const int SG = a.pn.S * a.pn.G;
    const int pst = a.pn.G * a.pn.rp * VW;
    Carve cv{smem};
    double *xs = cv.take<double>((size_t)NC * SG);
    double *part = cv.take<double>((size_t)NC * pst);
    double *redn = cv.take<double>((size_t)NC * NT);
    double *red2n = cv.take<double>((size_t)NC * 64);
    bool nodir = MODE == PAIR_TOP;   // as in pair_body: zero Dirichlet data for every component
#pragma unroll
    for (int c = 0; c < NC; ++c) nodir = nodir && !A.c[c].dir;
    const int s0 = nodir ? a.n12t / a.pn.G : 0;
    PanelStream<double, PF, UNR> ps;
    ps.start(reinterpret_cast<const double *>(a.pn.data) + (int64_t)node * a.pn.node_elems +
                 (int64_t)tile * a.pn.tile_elems + (int64_t)s0 * a.pn.rp * a.pn.G * VW,
             a.pn.rp, a.pn.G, a.pn.S - s0);
    const int rows = a.pn.rp * VW;
    const int myrow = tile * rows + threadIdx.x;
    const int64_t gbase = MODE == PAIR_TOP ? 0 : (int64_t)node * 4 * a.nbcc;
    const int *tab = a.tab;
    int kind = -1, idx = 0, p1 = -1, p2 = -1;
    double base[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) base[c] = 0.0;
    if ((int)threadIdx.x < rows && myrow < a.R) {
        if (MODE == PAIR_UP) {
            kind = tab[a.t_fin + 3 * myrow];
            idx = tab[a.t_fin + 3 * myrow + 1];
            if (kind == 2) {
                const int pass = tab[a.t_fin + 3 * myrow + 2];
#pragma unroll
                for (int c = 0; c < NC; ++c) base[c] = A.c[c].hg[gbase + pass];
            }
        } else {
            kind = tab[a.t_fin + 4 * myrow];
            idx = tab[a.t_fin + 4 * myrow + 1];
            p1 = tab[a.t_fin + 4 * myrow + 2];
            p2 = tab[a.t_fin + 4 * myrow + 3];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (kind == 1) base[c] = A.c[c].w3_t[(int64_t)node * a.n3t + idx];
                else if (kind == 0) base[c] = A.c[c].w3_c[(int64_t)node * 2 * a.n3c + idx];
            }
        }
    }
    for (int k = threadIdx.x; k < SG; k += NT) {
        double x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = 0.0;
        if (k < a.C) {
            if (MODE == PAIR_DOWN) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    x[c] = k < a.n12t ? A.c[c].ub_t[(int64_t)node * a.n12t + k]
                                      : A.c[c].w3_t[(int64_t)node * a.n3t + k - a.n12t];
            } else if (MODE == PAIR_TOP && k < a.n12t) {
                const int rm = a.root_map[k];
#pragma unroll
                for (int c = 0; c < NC; ++c) x[c] = A.c[c].dir ? A.c[c].dir[rm] : 0.0;
            } else {
                const int tp = tab[a.t_plus + k], tm = tab[a.t_minus + k];
                const int jc = tab[a.t_j3 + k];
                const int64_t j = jc >= 0 ? a.j3i_c[(int64_t)node * 2 * a.n3c + jc] : a.j3i_t[(int64_t)node * a.n3t - jc - 1];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    x[c] = A.c[c].hg[gbase + tp] - A.c[c].hg[gbase + tm];
                    if (A.c[c].r3) x[c] += A.c[c].r3[j];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) xs[c * SG + k] = x[c];
    }
    if (MODE != PAIR_UP) {
        const int per = (a.n12t + ntile - 1) / ntile;
        const int m1 = min(a.n12t, (tile + 1) * per);
        for (int m = tile * per + threadIdx.x; m < m1; m += NT) {
            const int dst = tab[a.t_copy + m];
            const int rm = MODE == PAIR_TOP ? a.root_map[m] : 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double v = MODE == PAIR_DOWN ? A.c[c].ub_t[(int64_t)node * a.n12t + m]
                                                   : (A.c[c].dir ? A.c[c].dir[rm] : 0.0);
                A.c[c].ubg[gbase + dst] = v;
            }
        }
    }
    __syncthreads();
    ps.template finish_n<NC>(xs + s0 * a.pn.G, SG, part, pst);
    __syncthreads();
    const int G = a.pn.G;
    const int nsl = min(G, NT / rows);
    const int t = threadIdx.x;
    const int row = t % rows, sl = t / rows;
    if (sl < nsl) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double y = 0.0;
            for (int gg = sl; gg < G; gg += nsl) y += part[c * pst + gg * rows + row];
            redn[c * NT + sl * rows + row] = y;
        }
    }
    __syncthreads();
    double y[NC];
    slice_sum_n<NC>(redn, NT, red2n, nsl, rows, y);
    if (t < rows && myrow < a.R) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const PairArgs &ac = A.c[c];
            if (MODE == PAIR_UP) {
                if (kind == 0) ac.w3_c[(int64_t)node * 2 * a.n3c + idx] = y[c];
                else if (kind == 1) ac.w3_t[(int64_t)node * a.n3t + idx] = y[c];
                else ac.h_t[(int64_t)node * a.n12t + idx] = base[c] + y[c];
            } else {
                const double u3 = y[c] + base[c];
                ac.ubg[gbase + p1] = u3;
                if (p2 >= 0) ac.ubg[gbase + p2] = u3;
            }
        }
    }
}

template <int NC, int MODE>
__global__ __launch_bounds__(NT) void k_pair_sys(PairArgsN<NC> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    pair_sys_body<NC, MODE>(a, blockIdx.x, smem);
}

// One composite product of several operators in one launch: workgroup w belongs to entry
// e, base[e] <= w < base[e + 1].
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_pair_group(const PairArgs *args, const int *base, int n) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    const int w = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    pair_body<T, MODE>(args[lo], w - base[lo], smem, red);
}

// =======================================================================================
// two-component level products (FP64): both components of one (node, row tile, column
// chunk) in one workgroup, the operator block streamed once for both
// =======================================================================================
template <int NC>
struct LevelSysArgsN {
    LevelArgs c[NC];   // per component (right-hand side); the operator fields are the same in all
};
using LevelSysArgs = LevelSysArgsN<2>;

// One (node, row tile, column chunk) of a level product for NC right-hand sides: the
// operator block is streamed once for all of them.  The input gathers of all components
// share one chain of index loads, and the row sums of all components share their barriers;
// every component's arithmetic is that of level_body, in the same order.
template <int NC, bool UP, int PFX = PF, int UNRX = UNR>
__device__ __forceinline__ void level_sys_body(const LevelSysArgsN<NC> &A, int blk, unsigned char *smem, double *red,
                                               int *s_last) {
    constexpr int VW = 2;
    const LevelArgs &a = A.c[0];
    const int kch = a.pn.kch, ntile = a.pn.ntile;
    const int chunk = blk % kch;
    const int tile = (blk / kch) % ntile;
    const int node = blk / (kch * ntile);
    const int SG = a.pn.S * a.pn.G;
    const int pst = a.pn.G * a.pn.rp * VW;
    Carve cv{smem};
    double *xs = cv.take<double>((size_t)NC * SG);
    double *part = cv.take<double>((size_t)NC * pst);
    double *redn = cv.take<double>((size_t)NC * NT);   // slice partials of every component
    double *red2n = cv.take<double>((size_t)NC * 64);  // their group sums
    PanelStream<double, PFX, UNRX> ps;
    ps.start(reinterpret_cast<const double *>(a.pn.data) + (int64_t)node * a.pn.node_elems +
                 (int64_t)(tile * kch + chunk) * a.pn.tile_elems,
             a.pn.rp, a.pn.G, a.pn.S);
    const int rows = a.pn.rp * VW;
    const int myrow = tile * rows + threadIdx.x;
    double fin[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) fin[c] = 0.0;
    int64_t ia = -1, ib = -1;
    if (kch == 1 && (int)threadIdx.x < rows) {
        if (UP) {
            if (!a.root && myrow >= a.n3 && myrow < a.n3 + a.n12) {
                const int m = myrow - a.n3;
                const int64_t at = (m < a.n1) ? (int64_t)(2 * node) * a.nbc + a.a1[m]
                                              : (int64_t)(2 * node + 1) * a.nbc + a.b2[m - a.n1];
#pragma unroll
                for (int c = 0; c < NC; ++c) fin[c] = A.c[c].hc[at];
            }
        } else if (myrow < a.n3) {
#pragma unroll
            for (int c = 0; c < NC; ++c) fin[c] = A.c[c].w3[(int64_t)node * a.n3 + myrow];
            ia = (int64_t)(2 * node) * a.nbc + a.a3[myrow];
            ib = (int64_t)(2 * node + 1) * a.nbc + a.b3[myrow];
        }
    }
    const int cols = UP ? a.n3 : a.n12;
    for (int k = threadIdx.x; k < SG; k += NT) {
        const int kg = chunk * SG + k;
        double x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = 0.0;
        if (kg < cols) {
            if (UP) {
                const int64_t pb = (int64_t)(2 * node + 1) * a.nbc + a.b3[kg];
                const int64_t pa = (int64_t)(2 * node) * a.nbc + a.a3[kg];
                const int64_t j = a.j3i[(int64_t)node * a.n3 + kg];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    x[c] = A.c[c].hc[pb] - A.c[c].hc[pa];
                    if (A.c[c].r3) x[c] += A.c[c].r3[j];
                }
            } else if (a.root) {
                const int rm = a.root_map[kg];
#pragma unroll
                for (int c = 0; c < NC; ++c) x[c] = A.c[c].dir ? A.c[c].dir[rm] : 0.0;
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) x[c] = A.c[c].ub[(int64_t)node * a.n12 + kg];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) xs[c * SG + k] = x[c];
    }
    if (!UP) {
        // the J1 / J2 parts of the children's boundary data are the parent's own; the
        // workgroups of the node copy one slice each
        const int nblk_node = ntile * kch, me = tile * kch + chunk;
        const int per = (a.n12 + nblk_node - 1) / nblk_node;
        const int m1 = min(a.n12, (me + 1) * per);
        for (int m = me * per + threadIdx.x; m < m1; m += NT) {
            const int64_t dst = (m < a.n1) ? (int64_t)(2 * node) * a.nbc + a.a1[m]
                                           : (int64_t)(2 * node + 1) * a.nbc + a.b2[m - a.n1];
            const int rm = a.root ? a.root_map[m] : 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const LevelArgs &ac = A.c[c];
                const double v = a.root ? (ac.dir ? ac.dir[rm] : 0.0) : ac.ub[(int64_t)node * a.n12 + m];
                ac.ubc[dst] = v;
            }
        }
    }
    __syncthreads();
    ps.template finish_n<NC>(xs, SG, part, pst);
    __syncthreads();
    if (kch == 1) {
        const int G = a.pn.G;
        const int nsl = min(G, NT / rows);
        const int t = threadIdx.x;
        const int row = t % rows, sl = t / rows;
        if (sl < nsl) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double y = 0.0;
                for (int gg = sl; gg < G; gg += nsl) y += part[c * pst + gg * rows + row];
                redn[c * NT + sl * rows + row] = y;
            }
        }
        __syncthreads();
        double y[NC];
        slice_sum_n<NC>(redn, NT, red2n, nsl, rows, y);
        if (t < rows) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const LevelArgs &ac = A.c[c];
                if (UP) {
                    if (myrow < a.n3) ac.w3[(int64_t)node * a.n3 + myrow] = y[c];
                    else if (!a.root && myrow < a.n3 + a.n12) ac.h[(int64_t)node * a.n12 + myrow - a.n3] = fin[c] + y[c];
                } else if (myrow < a.n3) {
                    const double u3 = y[c] + fin[c];
                    ac.ubc[ia] = u3;
                    ac.ubc[ib] = u3;
                }
            }
        }
        return;
    }
    // split-K: publish both components' partial sums; the last workgroup of the (node,
    // tile) to arrive (counted on component 0's counters) adds the chunks in a fixed order
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double *pp = A.c[c].part + ((int64_t)node * ntile + tile) * kch * rows;
        for (int idx = threadIdx.x; idx < rows; idx += NT)
            pp[(int64_t)chunk * rows + idx] = panel_sum<double>(part + c * pst, a.pn.rp, a.pn.G, idx);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *s_last = (atomicAdd(&a.cnt[node * ntile + tile], 1) == kch - 1);
    __syncthreads();
    if (!*s_last) return;
    __threadfence();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const LevelArgs &ac = A.c[c];
        const double *pp = ac.part + ((int64_t)node * ntile + tile) * kch * rows;
        for (int r0 = 0; r0 < rows; r0 += NT) {
            const int nr = min(NT, rows - r0);
            const int nsl = NT / nr;
            const int t = threadIdx.x;
            const int row = t % nr, sl = t / nr;
            if (sl < nsl) {
                double y = 0.0;
                for (int cc = sl; cc < kch; cc += nsl) y += pp[(int64_t)cc * rows + r0 + row];
                red[sl * nr + row] = y;
            }
            __syncthreads();
            if (t < nr) {
                double y = 0.0;
                for (int s2 = 0; s2 < nsl; ++s2) y += red[s2 * nr + t];
                if (UP) up_finalize(ac, node, tile * rows + r0 + t, y);
                else down_finalize(ac, node, tile * rows + r0 + t, y);
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) a.cnt[node * ntile + tile] = 0;
}

template <int NC, bool UP>
__global__ __launch_bounds__(NT) void k_level_sys(LevelSysArgsN<NC> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    __shared__ int s_last;
    level_sys_body<NC, UP>(a, blockIdx.x, smem, red, &s_last);
}

// Panels with S <= PF_SMALL: the same products with fewer registers.
template <int NC, bool UP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_level_sys_small(
    LevelSysArgsN<NC> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    __shared__ int s_last;
    level_sys_body<NC, UP, PF_SMALL, PF_SMALL>(a, blockIdx.x, smem, red, &s_last);
}

// =======================================================================================
// stage-1 evaluation (L u^n, F_1) and the refinement residual, from a canonical vector
// =======================================================================================
struct EvalArgs {
    LeafGeo geo;
    const double *u;
    const double *D, *D2, *coef;
    double *Lu;                 // L u at interior nodes, or null
    // residual mode
    const double *rhs;
    double gamma_dt;
    double *r_int, *flux;
};

// leaf cl in canonical order (cl = j*n1 + i), one workgroup.  Every global load (D, D2,
// the leaf's values, the first node's coefficients and right-hand side) is issued before
// the one barrier.  The tile's corners are never read (no mixed derivative), so they are
// not filled.
__device__ __forceinline__ void eval_body(const EvalArgs &a, int cl, double *tile, double *D, double *D2) {
    const int li = cl % a.geo.n1, lj = cl / a.geo.n1;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, ld = dmat_ld(p);
    const int64_t n_int = a.geo.n_int;
    const int64_t base = (int64_t)cl * q2;
    load_dmat_ld(a.D, D, p);
    load_dmat_ld(a.D2, D2, p);
    for (int k = threadIdx.x; k < q2; k += NT) tile[(k / q + 1) * p + (k % q) + 1] = a.u[base + k];
    for (int k = threadIdx.x; k < 4 * q; k += NT) {
        const int e = k / q, m = k % q;
        tile[edge_tile_pos(p, q, e, m)] = a.u[edge_index(a.geo, li, lj, e, m)];
    }
    const bool res = a.rhs != nullptr;
    double cf[5] = {0, 0, 0, 0, 0}, rh = 0.0;
    auto node_data = [&](int k) {
        const int64_t gi = base + k;
#pragma unroll
        for (int c = 0; c < 5; ++c) cf[c] = a.coef[c * n_int + gi];
        if (res) rh = a.rhs[gi];
    };
    if ((int)threadIdx.x < q2) node_data(threadIdx.x);
    __syncthreads();
    for (int k = threadIdx.x; k < q2; k += NT) {
        if (k != (int)threadIdx.x) node_data(k);
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
        const int64_t gi = base + k;
        if (res) {
            // refinement residual of (I - gamma_dt L) u = rhs at interior nodes
            a.r_int[gi] = rh - fma(-a.gamma_dt, Lu, u);
        } else if (a.Lu) {
            a.Lu[gi] = Lu;
        }
    }
    if (a.flux) {
        // coordinate-direction fluxes on the four leaf edges, [leaf][e][m]
        for (int k = threadIdx.x; k < 4 * q; k += NT) {
            const int e = k / q, m = k % q;
            const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * ld);
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

__global__ __launch_bounds__(NT) void k_eval(EvalArgs a) {
    __shared__ double tile[PMAX * PMAX];
    __shared__ double D[PMAX * dmat_ld(PMAX)], D2[PMAX * dmat_ld(PMAX)];
    eval_body(a, blockIdx.x, tile, D, D2);
}

// interface residual r3 = jump - (flux_alpha - flux_beta), interface-indexed
__device__ __forceinline__ void jump_body(const LeafGeo &g, const double *flux, const double *jump, double scale,
                                          double *r3, int64_t t) {
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
    r3[t] = scale * ((jump ? jump[t] : 0.0) - (fa - fb));
}

__global__ void k_jump(LeafGeo g, const double *flux, const double *jump, double scale, double *r3,
                       int64_t n_iface) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_iface) jump_body(g, flux, jump, scale, r3, t);
}

struct JumpArgs {
    LeafGeo g;
    const double *flux, *jump;
    double scale;
    double *r3;
    int64_t n_iface;
};

// first entry e with base[e] <= w < base[e + 1] (bisection)
__device__ __forceinline__ int group_entry(const int *base, int n, int w) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// the refinement residuals of several operators, in two launches (the jumps read the edge
// fluxes the evaluations write): leaf evaluations (workgroup w -> leaf w - ebase[e] of
// problem e), then the interface jumps (thread -> interface node of problem e by jbase)
__global__ __launch_bounds__(NT) void k_eval_group(const EvalArgs *ev, const int *ebase, int n) {
    __shared__ double tile[PMAX * PMAX];
    __shared__ double D[PMAX * dmat_ld(PMAX)], D2[PMAX * dmat_ld(PMAX)];
    const int w = blockIdx.x;
    const int e = group_entry(ebase, n, w);
    eval_body(ev[e], w - ebase[e], tile, D, D2);
}

__global__ void k_jump_group(const JumpArgs *jp, const int *jbase, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= jbase[n]) return;
    const int e = group_entry(jbase, n, t);
    const JumpArgs &j = jp[e];
    jump_body(j.g, j.flux, j.jump, j.scale, j.r3, t - jbase[e]);
}

// max over the leaves of a refinement pass's per-leaf max|delta| and max|u| (one workgroup;
// max is exact, so the order does not matter)
__device__ __forceinline__ void norm_fold_body(const NormFold &f) {
    __shared__ double wm[2][NT / 64];
    double d = 0.0, u = 0.0;
    for (int i = threadIdx.x; i < f.leaves; i += NT) {
        d = fmax(d, f.part[2 * i]);
        u = fmax(u, f.part[2 * i + 1]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        d = fmax(d, __shfl_xor(d, off));
        u = fmax(u, __shfl_xor(u, off));
    }
    if ((threadIdx.x & 63) == 0) {
        wm[0][threadIdx.x >> 6] = d;
        wm[1][threadIdx.x >> 6] = u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NT / 64; ++w) {
            d = fmax(d, wm[0][w]);
            u = fmax(u, wm[1][w]);
        }
        // non-negative doubles order like their bit patterns
        f.out[0] = (unsigned long long)__double_as_longlong(d);
        f.out[1] = (unsigned long long)__double_as_longlong(u);
    }
}

__global__ __launch_bounds__(NT) void k_norm_fold(NormFold f) { norm_fold_body(f); }

__global__ __launch_bounds__(NT) void k_norm_fold_group(const NormFold *folds) { norm_fold_body(folds[blockIdx.x]); }

__global__ void k_memop_group(const MemOp *ops, const int64_t *base, int n) {
    const int64_t total = base[n];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (base[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int64_t i = t - base[lo];
        double *d = reinterpret_cast<double *>(ops[lo].dst);
        d[i] = ops[lo].src ? reinterpret_cast<const double *>(ops[lo].src)[i] : 0.0;
    }
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
    const double *fpart;      // interior flux parts [leaf][4][q] (canonical leaf order)
    const double *D;          // p*p
    const double *cp;         // Thomas factors: cp[k], k = 1..nmax-1
    const double *inv_den;    // 1 / (diag - lower cp[k-1])
    const double *jump;       // flux_alpha - flux_beta per interface node (interface order) or null
    // the LDS kernel: the lines' end values come from the boundary data (f[ends[2t]],
    // f[ends[2t+1]], zero without f), and its workgroups also write all nb boundary values
    // of u (u[bnd_glob[k]] = f[k]) -- the boundary scatter in the same launch
    const double *f;
    const int *ends, *bnd_glob;
    int64_t nb;
};

// The arithmetic of one line system, shared by both line kernels so that they give the
// same bits: right-hand side of equation k, forward elimination, back substitution.
__device__ __forceinline__ double line_rhs(double fl, double fh, const double *jump, int64_t jidx, int k, int n,
                                           double lower, double upper, double e0, double en) {
    double r = fl - fh;
    if (jump) r += jump[jidx];
    if (k == 1) r -= lower * e0;
    if (k == n - 1) r -= upper * en;
    return r;
}

__device__ __forceinline__ double line_fwd(double r, int k, double lower, double dprev, double id) {
    return (r - (k > 1 ? lower * dprev : 0.0)) * id;
}

__device__ __forceinline__ double line_bwd(double dv, double cv, double enext) { return dv - cv * enext; }

// Geometry of line system t: orientation, length n, strides of u, flux parts and jumps.
struct LineGeo {
    int n;
    int64_t u0, ustride, l0, lstride, j0, jstride;
    int elo, ehi;
};

__device__ __forceinline__ bool line_geo(const LeafGeo &g, int t, LineGeo &L) {
    const int q = g.q;
    const int nvs = g.n2 * q;   // systems along horizontal rows (vertical-edge unknowns)
    const int nhs = g.n1 * q;
    if (t >= nvs + nhs) return false;
    const bool vert = t < nvs;
    L.n = vert ? g.n1 : g.n2;
    if (L.n < 2) return false;
    const int line = vert ? t / q : (t - nvs) / q;   // leaf row j (vert) or column i (horz)
    const int m0 = (vert ? t : t - nvs) % q;          // local node index along the edge
    L.ustride = vert ? (int64_t)g.n2 * q : (int64_t)g.n1 * q;
    L.u0 = vert ? g.n_int + (int64_t)line * q + m0 : g.n_int + g.n_vert + (int64_t)line * q + m0;
    // leaf number k along the line, flux part on side e
    L.lstride = vert ? 4 * q : (int64_t)g.n1 * 4 * q;
    L.l0 = (vert ? (int64_t)line * g.n1 * 4 * q : (int64_t)line * 4 * q) + m0;
    L.elo = vert ? 0 : 2;   // left/right or bottom/top sides
    L.ehi = vert ? 1 : 3;
    // interface index of the node on grid line k: vertical edges first, by line k-1
    L.j0 = vert ? (int64_t)line * q + m0 : (int64_t)(g.n1 - 1) * g.n2 * q + (int64_t)line * q + m0;
    L.jstride = vert ? (int64_t)g.n2 * q : (int64_t)g.n1 * q;
    return true;
}

// One thread per grid line; the recursion carries d_{k-1} and e_{k+1} in registers and
// its inputs are loaded CH at a time ahead of use, so no load waits on a store.
__device__ __forceinline__ void line_body(const LineArgs &a, int t) {
    constexpr int CH = 8;
    const LeafGeo &g = a.geo;
    const int p = g.p;
    LineGeo L;
    if (!line_geo(g, t, L)) return;
    const int n = L.n;
    const double *__restrict__ fpart = a.fpart;
    const double *__restrict__ cp = a.cp;
    const double *__restrict__ inv_den = a.inv_den;
    double *__restrict__ u = a.u;
    const double lower = a.D[(p - 1) * p + 0];
    const double upper = -a.D[0 * p + (p - 1)];
    const double e0 = u[L.u0], en = u[L.u0 + (int64_t)n * L.ustride];
    double dprev = 0.0;
    for (int k0 = 1; k0 < n; k0 += CH) {
        double fl[CH], fh[CH], id[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int k = k0 + c;
            if (k < n) {
                fl[c] = fpart[L.l0 + k * L.lstride + L.elo * g.q];
                fh[c] = fpart[L.l0 + (k - 1) * L.lstride + L.ehi * g.q];
                id[c] = inv_den[k];
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int k = k0 + c;
            if (k < n) {
                const double r = line_rhs(fl[c], fh[c], a.jump, L.j0 + (int64_t)(k - 1) * L.jstride, k, n, lower,
                                          upper, e0, en);
                const double d = line_fwd(r, k, lower, dprev, id[c]);
                u[L.u0 + k * L.ustride] = d;
                dprev = d;
            }
        }
    }
    double enext = dprev;   // e_{n-1} = d_{n-1}
    for (int k0 = n - 2; k0 >= 1; k0 -= CH) {
        double dv[CH], cv[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int k = k0 - c;
            if (k >= 1) {
                dv[c] = u[L.u0 + k * L.ustride];
                cv[c] = cp[k];
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int k = k0 - c;
            if (k >= 1) {
                enext = line_bwd(dv[c], cv[c], enext);
                u[L.u0 + k * L.ustride] = enext;
            }
        }
    }
}

// LINES lines per workgroup of LINE_NT threads: all waves first load the lines' right-hand
// sides (every equation of every line at once, no dependent chain) into LDS, then one
// thread per line runs the recursion out of LDS and writes only the final values.
constexpr int LINES = 16;
constexpr int LINE_NT = 256;

__global__ __launch_bounds__(LINE_NT) void k_interface_lines_lds(LineArgs a, int nmax) {
    extern __shared__ __align__(16) double lsm[];
    double *rr = lsm;                                  // [nmax][LINES]: r_k, then d_k
    double *sid = lsm + (size_t)nmax * LINES;          // [nmax]: 1 / den_k
    double *scp = sid + nmax;                          // [nmax]: cp_k
    const LeafGeo &g = a.geo;
    const int p = g.p;
    const int lane = threadIdx.x % LINES, wv = threadIdx.x / LINES;
    constexpr int NW = LINE_NT / LINES;
    const int t = blockIdx.x * LINES + lane;
    LineGeo L;
    const bool on = line_geo(g, t, L);
    const double lower = a.D[(p - 1) * p + 0];
    const double upper = -a.D[0 * p + (p - 1)];
    for (int k = threadIdx.x; k < nmax; k += LINE_NT) {
        sid[k] = a.inv_den[k];
        scp[k] = a.cp[k];
    }
    // the boundary values of u, a slice per workgroup
    {
        const int64_t per = (a.nb + gridDim.x - 1) / gridDim.x;
        const int64_t k1 = min(a.nb, (int64_t)(blockIdx.x + 1) * per);
        for (int64_t k = (int64_t)blockIdx.x * per + threadIdx.x; k < k1; k += LINE_NT)
            a.u[a.bnd_glob[k]] = a.f ? a.f[k] : 0.0;
    }
    double e0 = 0.0, en = 0.0;
    if (on) {
        e0 = a.f ? a.f[a.ends[2 * t]] : 0.0;
        en = a.f ? a.f[a.ends[2 * t + 1]] : 0.0;
        for (int k = 1 + wv; k < L.n; k += NW)
            rr[k * LINES + lane] = line_rhs(a.fpart[L.l0 + k * L.lstride + L.elo * g.q],
                                            a.fpart[L.l0 + (k - 1) * L.lstride + L.ehi * g.q], a.jump,
                                            L.j0 + (int64_t)(k - 1) * L.jstride, k, L.n, lower, upper, e0, en);
    }
    __syncthreads();
    if (wv != 0 || !on) return;
    const int n = L.n;
    double dprev = 0.0;
    for (int k = 1; k < n; ++k) {
        const double d = line_fwd(rr[k * LINES + lane], k, lower, dprev, sid[k]);
        rr[k * LINES + lane] = d;
        dprev = d;
    }
    double enext = dprev;   // e_{n-1} = d_{n-1}
    a.u[L.u0 + (int64_t)(n - 1) * L.ustride] = enext;
    for (int k = n - 2; k >= 1; --k) {
        enext = line_bwd(rr[k * LINES + lane], scp[k], enext);
        a.u[L.u0 + k * L.ustride] = enext;
    }
}

// 64 threads per workgroup: each thread carries a whole line system in registers
__global__ __launch_bounds__(64) void k_interface_lines(LineArgs a) {
    line_body(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// Line systems of several operators: thread index t belongs to problem b,
// base[b] <= t < base[b + 1]; then the outer-boundary data of each problem (zero).
__global__ __launch_bounds__(64) void k_lines_group(const LineArgs *args, const int *base, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= base[n]) return;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    line_body(args[lo], t - base[lo]);
}

struct ScatterTask {
    const int *bnd_glob;
    double *u;
};

__global__ void k_zero_boundary_group(const ScatterTask *tasks, const int *base, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= base[n]) return;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    tasks[lo].u[tasks[lo].bnd_glob[t - base[lo]]] = 0.0;
}

// up to 8 host values handed over as a kernel argument (no host buffer stays in use)
struct Values8 {
    double v[8];
};

__global__ void k_set_values(double *dst, Values8 v, int n) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = v.v[threadIdx.x];
}

__global__ void k_zero(double *p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0.0;
}

__global__ void k_copy(double *dst, const double *src, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

// ---- profiling ---------------------------------------------------------------------------
const char *const kKernelFamilyNames[KF_COUNT] = {
    "leaf_up_fp64", "leaf_up_fp32", "leaf_down_fp64", "leaf_down_fp32", "leaf_eval_up_fp64",
    "leaf_eval_up_fp32", "leaf_down_up_fp64", "leaf_down_up_fp32", "leaf_down_update_fp64",
    "leaf_eval_update", "level_up_fp64", "level_up_fp32", "level_down_fp64", "level_down_fp32",
    "residual", "lines", "leaf2_eval_up_fp64", "leaf2_down_up_fp64", "leaf2_down_update_fp64",
    "level2_up_fp64", "level2_down_fp64", "leafc_eval_up_fp64", "leafc_down_up_fp64", "leafc_down_update_fp64",
    "leafc_solve_fp64", "pair_up_fp64", "pair_top_fp64", "pair_down_fp64", "pair_up_fp32", "pair_top_fp32",
    "pair_down_fp32", "direct_fp64"};

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


// =======================================================================================
// launchers
// =======================================================================================
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
    a.cnt = up ? (fp32 ? L.cnt_up32 : L.cnt_up64) : (fp32 ? L.cnt_dn32 : L.cnt_dn64);
    return a;
}

// The root's upward and downward products in one kernel: with u_12 the Dirichlet data,
// u_3 = S u_12 + X d needs, for each row tile, only that tile's rows of X and of S.
template <typename T>
__device__ __forceinline__ void root_body(const LevelArgs &up, const LevelArgs &dn, int tile, unsigned char *smem,
                                          double *red) {
    constexpr int VW = 16 / sizeof(T);
    const int SG1 = up.pn.S * up.pn.G, SG2 = dn.pn.S * dn.pn.G;
    Carve cv{smem};
    T *xs1 = cv.take<T>(SG1);
    T *xs2 = cv.take<T>(SG2);
    T *part1 = cv.take<T>((size_t)up.pn.G * up.pn.rp * VW);
    T *part2 = cv.take<T>((size_t)dn.pn.G * dn.pn.rp * VW);
    // both operators' first loads are issued before the inputs are gathered; without
    // Dirichlet data S u_12 is zero and S is not read (the sum of its zero products is +0,
    // so u_3 = 0 + X d is the same either way)
    const bool with_s = dn.dir != nullptr;
    PanelStream<T, PF, UNR> ps, ps2;
    ps.start(reinterpret_cast<const T *>(up.pn.data) + (int64_t)tile * up.pn.tile_elems, up.pn.rp, up.pn.G, up.pn.S);
    if (with_s)
        ps2.start(reinterpret_cast<const T *>(dn.pn.data) + (int64_t)tile * dn.pn.tile_elems, dn.pn.rp, dn.pn.G,
                  dn.pn.S);
    const int rows = up.pn.rp * VW;   // the same row tiling for X and S
    const int myrow = tile * rows + threadIdx.x;
    int64_t ia = -1, ib = -1;
    if ((int)threadIdx.x < rows && myrow < dn.n3) {
        ia = dn.a3[myrow];
        ib = (int64_t)dn.nbc + dn.b3[myrow];
    }
    for (int k = threadIdx.x; k < SG1; k += NT) {
        double x = 0.0;
        if (k < up.n3) {
            x = up.hc[(int64_t)up.nbc + up.b3[k]] - up.hc[up.a3[k]];
            if (up.r3) x += up.r3[up.j3i[k]];
        }
        xs1[k] = (T)x;
    }
    for (int k = threadIdx.x; k < SG2; k += NT)
        xs2[k] = (T)((k < dn.n12 && dn.dir) ? dn.dir[dn.root_map[k]] : 0.0);
    {   // the children's J1 / J2 boundary data: one slice per workgroup
        const int per = (dn.n12 + dn.pn.ntile - 1) / dn.pn.ntile;
        const int m1 = min(dn.n12, (tile + 1) * per);
        for (int m = tile * per + threadIdx.x; m < m1; m += NT) {
            const double v = dn.dir ? dn.dir[dn.root_map[m]] : 0.0;
            if (m < dn.n1) dn.ubc[dn.a1[m]] = v;
            else dn.ubc[(int64_t)dn.nbc + dn.b2[m - dn.n1]] = v;
        }
    }
    __syncthreads();
    ps.finish(xs1, part1);
    if (with_s) ps2.finish(xs2, part2);
    __syncthreads();
    // deterministic sums over the column groups of both products, then u_3 = S u_12 + X d
    const int nsl1 = min(up.pn.G, NT / rows), nsl2 = min(dn.pn.G, NT / rows);
    const int t = threadIdx.x, row = t % rows, sl = t / rows;
    double y1 = 0.0, y2 = 0.0;
    if (sl < nsl1) {
        T y = T(0);
        for (int gg = sl; gg < up.pn.G; gg += nsl1) y += part1[gg * rows + row];
        y1 = (double)y;
    }
    if (with_s && sl < nsl2) {
        T y = T(0);
        for (int gg = sl; gg < dn.pn.G; gg += nsl2) y += part2[gg * rows + row];
        y2 = (double)y;
    }
    red[t] = y1;
    __syncthreads();
    const double w3 = slice_sum(red, red + NT, nsl1, rows);
    __syncthreads();
    red[t] = y2;
    __syncthreads();
    const double su = slice_sum(red, red + NT, nsl2, rows);
    if (t < rows && myrow < dn.n3) {
        const double u3 = su + w3;
        dn.ubc[ia] = u3;
        dn.ubc[ib] = u3;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_root(LevelArgs up, LevelArgs dn) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    root_body<T>(up, dn, blockIdx.x, smem, red);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_root_group(const LevelArgs *ups, const LevelArgs *dns, const int *base,
                                                   int n) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    const int w = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    root_body<T>(ups[lo], dns[lo], w - base[lo], smem, red);
}

// The fused root for NC components: u_3 = S u_12 + X d for each.
template <int NC>
__device__ __forceinline__ void root_sys_body(const LevelSysArgsN<NC> &U, const LevelSysArgsN<NC> &Dn, int tile,
                                              unsigned char *smem, double *red) {
    constexpr int VW = 2;
    const LevelArgs &up = U.c[0], &dn = Dn.c[0];
    const int SG1 = up.pn.S * up.pn.G, SG2 = dn.pn.S * dn.pn.G;
    const int pst1 = up.pn.G * up.pn.rp * VW, pst2 = dn.pn.G * dn.pn.rp * VW;
    Carve cv{smem};
    double *xs1 = cv.take<double>((size_t)NC * SG1);
    double *xs2 = cv.take<double>((size_t)NC * SG2);
    double *part1 = cv.take<double>((size_t)NC * pst1);
    double *part2 = cv.take<double>((size_t)NC * pst2);
    PanelStream<double, PF, UNR> ps, ps2;
    ps.start(reinterpret_cast<const double *>(up.pn.data) + (int64_t)tile * up.pn.tile_elems, up.pn.rp, up.pn.G,
             up.pn.S);
    ps2.start(reinterpret_cast<const double *>(dn.pn.data) + (int64_t)tile * dn.pn.tile_elems, dn.pn.rp, dn.pn.G,
              dn.pn.S);
    const int rows = up.pn.rp * VW;
    const int myrow = tile * rows + threadIdx.x;
    int64_t ia = -1, ib = -1;
    if ((int)threadIdx.x < rows && myrow < dn.n3) {
        ia = dn.a3[myrow];
        ib = (int64_t)dn.nbc + dn.b3[myrow];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const LevelArgs &uc = U.c[c], &dc = Dn.c[c];
        for (int k = threadIdx.x; k < SG1; k += NT) {
            double x = 0.0;
            if (k < up.n3) {
                x = uc.hc[(int64_t)up.nbc + up.b3[k]] - uc.hc[up.a3[k]];
                if (uc.r3) x += uc.r3[up.j3i[k]];
            }
            xs1[c * SG1 + k] = x;
        }
        for (int k = threadIdx.x; k < SG2; k += NT)
            xs2[c * SG2 + k] = (k < dn.n12 && dc.dir) ? dc.dir[dn.root_map[k]] : 0.0;
        const int per = (dn.n12 + dn.pn.ntile - 1) / dn.pn.ntile;
        const int m1 = min(dn.n12, (tile + 1) * per);
        for (int m = tile * per + threadIdx.x; m < m1; m += NT) {
            const double v = dc.dir ? dc.dir[dn.root_map[m]] : 0.0;
            if (m < dn.n1) dc.ubc[dn.a1[m]] = v;
            else dc.ubc[(int64_t)dn.nbc + dn.b2[m - dn.n1]] = v;
        }
    }
    __syncthreads();
    ps.finish_n<NC>(xs1, SG1, part1, pst1);
    ps2.finish_n<NC>(xs2, SG2, part2, pst2);
    __syncthreads();
    const int nsl1 = min(up.pn.G, NT / rows), nsl2 = min(dn.pn.G, NT / rows);
    const int t = threadIdx.x, row = t % rows, sl = t / rows;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double y1 = 0.0, y2 = 0.0;
        if (sl < nsl1)
            for (int gg = sl; gg < up.pn.G; gg += nsl1) y1 += part1[c * pst1 + gg * rows + row];
        if (sl < nsl2)
            for (int gg = sl; gg < dn.pn.G; gg += nsl2) y2 += part2[c * pst2 + gg * rows + row];
        red[t] = y1;
        __syncthreads();
        const double w3 = slice_sum(red, red + NT, nsl1, rows);
        __syncthreads();
        red[t] = y2;
        __syncthreads();
        const double su = slice_sum(red, red + NT, nsl2, rows);
        if (t < rows && myrow < dn.n3) {
            const double u3 = su + w3;
            Dn.c[c].ubc[ia] = u3;
            Dn.c[c].ubc[ib] = u3;
        }
        __syncthreads();
    }
}

template <int NC>
__global__ __launch_bounds__(NT) void k_root_sys(LevelSysArgsN<NC> up, LevelSysArgsN<NC> dn) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    root_sys_body<NC>(up, dn, blockIdx.x, smem, red);
}

// The whole level sweep of a small tree as one product: interface values y = M h for the
// leaves' particular fluxes h (no boundary or jump data), each written to the two leaf
// boundary slots it belongs to, and zeros to the slots on the domain boundary.  One
// workgroup per row tile of M; the arithmetic of pair_body's product and row sums.
struct DirectArgs {
    PanelView pn;
    int R, C;
    const double *h;
    double *ub;
    const int *rows, *zero;
    int nzero;
};

// one row tile of the direct product (tile of ntiles); the tiles also clear the zero slots
__device__ __forceinline__ void direct_body(const DirectArgs &a, int tile, int ntiles, unsigned char *smem,
                                            double *red) {
    constexpr int VW = 2;
    const int SG = a.pn.S * a.pn.G;
    Carve cv{smem};
    double *xs = cv.take<double>(SG);
    double *part = cv.take<double>((size_t)a.pn.G * a.pn.rp * VW);
    PanelStream<double, PF, UNR> ps;
    ps.start(reinterpret_cast<const double *>(a.pn.data) + (int64_t)tile * a.pn.tile_elems, a.pn.rp, a.pn.G, a.pn.S);
    for (int k = threadIdx.x; k < SG; k += NT) xs[k] = k < a.C ? a.h[k] : 0.0;
    for (int z = tile * NT + threadIdx.x; z < a.nzero; z += ntiles * NT) a.ub[a.zero[z]] = 0.0;
    __syncthreads();
    ps.finish(xs, part);
    __syncthreads();
    const int rows = a.pn.rp * VW;
    const int G = a.pn.G;
    const int nsl = min(G, NT / rows);
    const int t = threadIdx.x;
    const int row = t % rows, sl = t / rows;
    if (sl < nsl) {
        double y = 0.0;
        for (int gg = sl; gg < G; gg += nsl) y += part[gg * rows + row];
        red[sl * rows + row] = y;
    }
    __syncthreads();
    const double y = slice_sum(red, red + NT, nsl, rows);
    const int myrow = tile * rows + t;
    if (t < rows && myrow < a.R) {
        a.ub[a.rows[2 * myrow]] = y;
        a.ub[a.rows[2 * myrow + 1]] = y;
    }
}

__global__ __launch_bounds__(NT) void k_direct(DirectArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    direct_body(a, blockIdx.x, gridDim.x, smem, red);
}

// several problems' direct products in one launch: base[b] is problem b's first workgroup
__global__ __launch_bounds__(NT) void k_direct_group(const DirectArgs *args, const int *base, int n) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT + 64];
    const int w = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    direct_body(args[lo], w - base[lo], base[lo + 1] - base[lo], smem, red);
}

static size_t level_lds(const Panel &pn) {
    const size_t es = pn.vw == 2 ? 8 : 4;
    return carve_bytes({(size_t)pn.S * pn.G * es, (size_t)pn.G * pn.rp * pn.vw * es});
}

static bool root_fusable(const hps_op *op, bool fp32) {
    if (op->L < 1) return false;
    const Panel &x = fp32 ? op->lv[0].xu32 : op->lv[0].xu64;
    const Panel &sp = fp32 ? op->lv[0].s32 : op->lv[0].s64;
    return x.kch == 1 && sp.kch == 1 && x.ntile == sp.ntile && x.rp == sp.rp &&
           level_lds(x) + level_lds(sp) <= 65536;
}

// single-leaf tree: the leaf boundary is the domain boundary
__global__ void k_root_leaf_ub(const double *dir, const int *root_map, double *ub, int nb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nb) ub[t] = dir ? dir[root_map[t]] : 0.0;
}

static void use_workspace(const hps_op *op, int l, bool up, const Workspace *ws, LevelArgs &a);

// FP64 sweeps through the composite level pairs: the top pair (root and level 1) in one
// launch, pairs (l, l + 1) for even l >= 2 one launch per direction, and an odd number of
// levels leaves the bottom level to the single-level kernels.
// The arguments of composite pair l's kernel (mode PAIR_UP / PAIR_DOWN / PAIR_TOP), on the
// operator's solve buffers or on workspace ws.
static PairArgs pair_args(const hps_op *op, int l, int mode, const double *jump, const double *dirichlet,
                          const Workspace *ws, bool fp32 = false) {
    const int L = op->L;
    auto hbuf = [&](int k) -> double * {
        if (k == L) return ws ? ws->h_leaf : op->h_leaf;
        return ws ? ws->lv[k].h : op->lv[k].h;
    };
    auto ubbuf = [&](int k) -> double * {
        if (k == L) return ws ? ws->ub_leaf : op->ub_leaf;
        return ws ? ws->lv[k].ub : op->lv[k].ub;
    };
    auto w3buf = [&](int k) -> double * { return ws ? ws->lv[k].w3 : op->lv[k].w3; };
    const bool up = (mode == PAIR_UP);
    const PairOps &P = op->pairs[l / 2];
    const Level &T = op->lv[l], &Cl = op->lv[l + 1];
    PairArgs a{};
    a.pn = view(up ? (fp32 ? P.up32 : P.up) : (fp32 ? P.dn32 : P.dn));
    a.R = up ? P.R_up : P.R_dn;
    a.C = up ? P.C_up : P.C_dn;
    a.n3t = T.n3;
    a.n12t = T.n12;
    a.n3c = Cl.n3;
    a.nbcc = Cl.nbc;
    a.tab = P.tab;
    a.t_plus = P.t_plus;
    a.t_minus = P.t_minus;
    a.t_j3 = P.t_j3;
    a.t_fin = up ? P.t_fin_up : P.t_fin_dn;
    a.t_copy = P.t_copy;
    a.hg = hbuf(l + 2);
    a.r3 = jump;
    a.j3i_t = T.j3i;
    a.j3i_c = Cl.j3i;
    a.h_t = hbuf(l);
    a.w3_t = w3buf(l);
    a.w3_c = w3buf(l + 1);
    a.ub_t = ubbuf(l);
    a.ubg = ubbuf(l + 2);
    a.dir = dirichlet;
    a.root_map = op->root_map;
    return a;
}

// The upper level of the lowest composite pair (an odd number of levels leaves the bottom
// level to the single-level kernels).
static int lowest_pair(const hps_op *op) { return (op->L % 2 == 1) ? op->L - 3 : op->L - 2; }

// FP64 sweeps through the composite level pairs: the top pair (root and level 1) in one
// launch, pairs (l, l + 1) for even l >= 2 one launch per direction, and an odd number of
// levels leaves the bottom level to the single-level kernels.
static int launch_pairs(const hps_op *op, bool fp32, const double *jump, const double *dirichlet, hipStream_t st,
                        const Workspace *ws) {
    const int L = op->L;
    auto single = [&](int l, bool up) {
        LevelArgs a = level_args(op, l, fp32, up);
        use_workspace(op, l, up, ws, a);
        a.r3 = jump;
        a.dir = dirichlet;
        const Panel &pn = up ? (fp32 ? op->lv[l].xu32 : op->lv[l].xu64) : (fp32 ? op->lv[l].s32 : op->lv[l].s64);
        const unsigned nb = (unsigned)(op->lv[l].nodes * a.pn.ntile * a.pn.kch);
        if (fp32) {
            if (up) launch_level<float, true>(a, nb, level_lds(pn), st);
            else launch_level<float, false>(a, nb, level_lds(pn), st);
        } else {
            if (up) launch_level<double, true>(a, nb, level_lds(pn), st);
            else launch_level<double, false>(a, nb, level_lds(pn), st);
        }
        HPS_LAUNCHED();
        return HPS_OK;
    };
    auto pair = [&](auto kern, int l, int mode) {
        const PairArgs a = pair_args(op, l, mode, jump, dirichlet, ws, fp32);
        const PairOps &P = op->pairs[l / 2];
        const Panel &pn = mode == PAIR_UP ? (fp32 ? P.up32 : P.up) : (fp32 ? P.dn32 : P.dn);
        hipLaunchKernelGGL(kern, dim3((unsigned)(op->lv[l].nodes * pn.ntile)), dim3(NT), level_lds(pn), st, a);
        HPS_LAUNCHED();
        return HPS_OK;
    };
    const int top_low = lowest_pair(op);
    {
        ProfScope ps_(&op->prof, fp32 ? KF_PAIR_UP32 : KF_PAIR_UP64, st);
        if (L % 2 == 1) TRY(single(L - 1, true));
        for (int l = top_low; l >= 2; l -= 2) {
            if (fp32) TRY(pair(k_pair<float, PAIR_UP>, l, PAIR_UP));
            else TRY(pair(k_pair<double, PAIR_UP>, l, PAIR_UP));
        }
    }
    {
        ProfScope ps_(&op->prof, fp32 ? KF_PAIR_TOP32 : KF_PAIR_TOP64, st);
        if (fp32) TRY(pair(k_pair<float, PAIR_TOP>, 0, PAIR_TOP));
        else TRY(pair(k_pair<double, PAIR_TOP>, 0, PAIR_TOP));
    }
    ProfScope ps_(&op->prof, fp32 ? KF_PAIR_DOWN32 : KF_PAIR_DOWN64, st);
    for (int l = 2; l <= top_low; l += 2) {
        if (fp32) TRY(pair(k_pair<float, PAIR_DOWN>, l, PAIR_DOWN));
        else TRY(pair(k_pair<double, PAIR_DOWN>, l, PAIR_DOWN));
    }
    if (L % 2 == 1) TRY(single(L - 1, false));
    return HPS_OK;
}

static DirectArgs direct_args(const hps_op *op, const Workspace *ws) {
    return DirectArgs{view(op->dpn),  op->dpn.R, op->dpn.C, ws ? ws->h_leaf : op->h_leaf, ws ? ws->ub_leaf : op->ub_leaf,
                      op->d_rows,     op->d_zero, op->n_zero};
}

int launch_direct(const hps_op *op, hipStream_t st, const Workspace *ws) {
    ProfScope ps_(&op->prof, KF_DIRECT64, st);
    hipLaunchKernelGGL(k_direct, dim3((unsigned)op->dpn.ntile), dim3(NT), level_lds(op->dpn), st,
                       direct_args(op, ws));
    HPS_LAUNCHED();
    return HPS_OK;
}

size_t direct_record_size() { return sizeof(DirectArgs); }

void direct_record(const hps_op *op, void *dst, int *blocks, size_t *lds, const Workspace *ws) {
    *reinterpret_cast<DirectArgs *>(dst) = direct_args(op, ws);
    *blocks = (int)op->dpn.ntile;
    *lds = level_lds(op->dpn);
}

int launch_direct_group(const void *args, const int *base, int n, int total, size_t lds, hipStream_t st) {
    if (total <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_direct_group, dim3(total), dim3(NT), lds, st, reinterpret_cast<const DirectArgs *>(args),
                       base, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_levels(const hps_op *op, bool fp32, const double *jump, const double *dirichlet, hipStream_t st,
                  const Workspace *ws) {
    if (op->direct && !fp32 && !jump && !dirichlet) return launch_direct(op, st, ws);
    if (op->composed) return launch_pairs(op, fp32, jump, dirichlet, st, ws);
    const bool rootf = root_fusable(op, fp32);
    {
        ProfScope ps_(&op->prof, fp32 ? KF_LEVEL_UP32 : KF_LEVEL_UP64, st);
        for (int l = op->L - 1; l >= (rootf ? 1 : 0); --l) {
            LevelArgs a = level_args(op, l, fp32, true);
            use_workspace(op, l, true, ws, a);
            a.r3 = jump;
            const Panel &pn = fp32 ? op->lv[l].xu32 : op->lv[l].xu64;
            const unsigned nb = (unsigned)(op->lv[l].nodes * a.pn.ntile * a.pn.kch);
            if (fp32) launch_level<float, true>(a, nb, level_lds(pn), st);
            else launch_level<double, true>(a, nb, level_lds(pn), st);
            HPS_LAUNCHED();
        }
    }
    ProfScope ps_(&op->prof, fp32 ? KF_LEVEL_DOWN32 : KF_LEVEL_DOWN64, st);
    if (op->L == 0) {
        hipLaunchKernelGGL(k_root_leaf_ub, dim3(1), dim3(NT), 0, st, dirichlet, (const int *)op->root_map,
                           ws ? ws->ub_leaf : op->ub_leaf, 4 * op->q * op->ncomp);
        HPS_LAUNCHED();
        return HPS_OK;
    }
    if (rootf) {
        LevelArgs up = level_args(op, 0, fp32, true), dn = level_args(op, 0, fp32, false);
        use_workspace(op, 0, true, ws, up);
        use_workspace(op, 0, false, ws, dn);
        up.r3 = jump;
        dn.dir = dirichlet;
        const Panel &x = fp32 ? op->lv[0].xu32 : op->lv[0].xu64;
        const Panel &sp = fp32 ? op->lv[0].s32 : op->lv[0].s64;
        const size_t lds = level_lds(x) + level_lds(sp) + 32;
        if (fp32) hipLaunchKernelGGL(k_root<float>, dim3(x.ntile), dim3(NT), lds, st, up, dn);
        else hipLaunchKernelGGL(k_root<double>, dim3(x.ntile), dim3(NT), lds, st, up, dn);
        HPS_LAUNCHED();
    }
    for (int l = rootf ? 1 : 0; l < op->L; ++l) {
        LevelArgs a = level_args(op, l, fp32, false);
        use_workspace(op, l, false, ws, a);
        a.dir = dirichlet;
        const Panel &pn = fp32 ? op->lv[l].s32 : op->lv[l].s64;
        const unsigned nb = (unsigned)(op->lv[l].nodes * a.pn.ntile * a.pn.kch);
        if (fp32) launch_level<float, false>(a, nb, level_lds(pn), st);
        else launch_level<double, false>(a, nb, level_lds(pn), st);
        HPS_LAUNCHED();
    }
    return HPS_OK;
}

// ---- two components on one operator (FP64) ----

static size_t sys_level_lds(const Panel &pn, int nc) {
    return carve_bytes({(size_t)nc * pn.S * pn.G * 8, (size_t)nc * pn.G * pn.rp * pn.vw * 8, (size_t)nc * NT * 8,
                        (size_t)nc * 64 * 8});
}

static size_t sys_root_lds(const hps_op *op, int nc) {
    const Panel &x = op->lv[0].xu64, &sp = op->lv[0].s64;
    return carve_bytes({(size_t)nc * x.S * x.G * 8, (size_t)nc * sp.S * sp.G * 8, (size_t)nc * x.G * x.rp * x.vw * 8,
                        (size_t)nc * sp.G * sp.rp * sp.vw * 8}) + 32;
}

// Dynamic LDS a multi-component level kernel may take on the current device (the kernels'
// static arrays take the rest).
static size_t sys_lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
        (void)hipGetLastError();
        return 65536 - 4096;
    }
    return (size_t)v - 4096;
}

bool levels_multi_fit(const hps_op *op, int nc) {
    const size_t lim = sys_lds_limit();
    for (int l = 0; l < op->L; ++l)
        if (sys_level_lds(op->lv[l].xu64, nc) > lim || sys_level_lds(op->lv[l].s64, nc) > lim) return false;
    return true;
}

// One level's product for NC right-hand sides (component c: workspace ws[c], Dirichlet
// data dir[c], interface jumps jump[c]; null: the operator's own / zero).
template <int NC>
static int level_multi_launch(const hps_op *op, int l, bool up, const Workspace *const *ws,
                              const double *const *dir, const double *const *jump, size_t lim, hipStream_t st) {
    const Panel &pn = up ? op->lv[l].xu64 : op->lv[l].s64;
    const unsigned nb = (unsigned)(op->lv[l].nodes * pn.ntile * pn.kch);
    // at most NC * XS_BYTES of input vectors plus the partial sums: within the LDS of a
    // gfx950 workgroup (160 KiB) for the sizes callers pass
    const size_t lds = sys_level_lds(pn, NC);
    if (lds > lim) {
        hps_set_error("%d-component level product needs %zu bytes of LDS, the device allows %zu", NC, lds, lim);
        return HPS_EDEVICE;
    }
    LevelSysArgsN<NC> A;
    for (int c = 0; c < NC; ++c) {
        A.c[c] = level_args(op, l, false, up);
        use_workspace(op, l, up, ws[c], A.c[c]);
        A.c[c].dir = dir ? dir[c] : nullptr;
        A.c[c].r3 = jump ? jump[c] : nullptr;
    }
    if (pn.S <= PF_SMALL) {
        if (up) hipLaunchKernelGGL((k_level_sys_small<NC, true>), dim3(nb), dim3(NT), lds, st, A);
        else hipLaunchKernelGGL((k_level_sys_small<NC, false>), dim3(nb), dim3(NT), lds, st, A);
    } else {
        if (up) hipLaunchKernelGGL((k_level_sys<NC, true>), dim3(nb), dim3(NT), lds, st, A);
        else hipLaunchKernelGGL((k_level_sys<NC, false>), dim3(nb), dim3(NT), lds, st, A);
    }
    HPS_LAUNCHED();
    return HPS_OK;
}

static size_t pair_sys_lds(const Panel &pn, int nc) {
    return carve_bytes({(size_t)nc * pn.S * pn.G * 8, (size_t)nc * pn.G * pn.rp * pn.vw * 8, (size_t)nc * NT * 8,
                        (size_t)nc * 64 * 8});
}

template <int K, int MODE>
static void pair_sys_launch(const hps_op *op, int l, const PairArgs *cs, hipStream_t st) {
    const Panel &pn = MODE == PAIR_UP ? op->pairs[l / 2].up : op->pairs[l / 2].dn;
    const unsigned nb = (unsigned)(op->lv[l].nodes * pn.ntile);
    if (K == 1) {   // the single-problem kernel (the same arithmetic, fewer registers)
        hipLaunchKernelGGL((k_pair<double, MODE>), dim3(nb), dim3(NT), level_lds(pn), st, cs[0]);
    } else {
        PairArgsN<K> A;
        for (int c = 0; c < K; ++c) A.c[c] = cs[c];
        hipLaunchKernelGGL((k_pair_sys<K, MODE>), dim3(nb), dim3(NT), pair_sys_lds(pn, K), st, A);
    }
}

// Composite pair l (mode PAIR_UP / PAIR_DOWN / PAIR_TOP) for components cs[0..n): as many
// components per launch as the LDS holds (the top pair's input vectors are the longest).
template <int MODE>
static int pair_multi_launch(const hps_op *op, int l, const PairArgs *cs, int n, size_t lim, hipStream_t st) {
    const Panel &pn = MODE == PAIR_UP ? op->pairs[l / 2].up : op->pairs[l / 2].dn;
    int k = n;
    while (k > 1 && pair_sys_lds(pn, k) > lim) --k;
    for (int c0 = 0; c0 < n; c0 += k) {
        switch (std::min(k, n - c0)) {
            case 1: pair_sys_launch<1, MODE>(op, l, cs + c0, st); break;
            case 2: pair_sys_launch<2, MODE>(op, l, cs + c0, st); break;
            case 3: pair_sys_launch<3, MODE>(op, l, cs + c0, st); break;
            default: pair_sys_launch<4, MODE>(op, l, cs + c0, st); break;
        }
        HPS_LAUNCHED();
    }
    return HPS_OK;
}

// The sweeps of an operator with composite pairs for NC right-hand sides: each composite
// (and the single bottom level of an odd tree) streamed once for all of them.
template <int NC>
static int pairs_multi(const hps_op *op, const Workspace *const *ws, const double *const *dir,
                       const double *const *jump, hipStream_t st, int fam_up, int fam_dn) {
    const size_t lim = sys_lds_limit();
    const int L = op->L, top_low = lowest_pair(op);
    PairArgs cs[NC];
    auto fill = [&](int l, int mode) {
        for (int c = 0; c < NC; ++c)
            cs[c] = pair_args(op, l, mode, jump ? jump[c] : nullptr, dir ? dir[c] : nullptr, ws[c]);
    };
    {
        ProfScope ps_(&op->prof, fam_up, st);
        if (L % 2 == 1) TRY(level_multi_launch<NC>(op, L - 1, true, ws, dir, jump, lim, st));
        for (int l = top_low; l >= 2; l -= 2) {
            fill(l, PAIR_UP);
            TRY(pair_multi_launch<PAIR_UP>(op, l, cs, NC, lim, st));
        }
    }
    ProfScope ps_(&op->prof, fam_dn, st);
    fill(0, PAIR_TOP);
    TRY(pair_multi_launch<PAIR_TOP>(op, 0, cs, NC, lim, st));
    for (int l = 2; l <= top_low; l += 2) {
        fill(l, PAIR_DOWN);
        TRY(pair_multi_launch<PAIR_DOWN>(op, l, cs, NC, lim, st));
    }
    if (L % 2 == 1) TRY(level_multi_launch<NC>(op, L - 1, false, ws, dir, jump, lim, st));
    return HPS_OK;
}

// The level sweeps of NC right-hand sides at once (FP64): every operator block is read
// once for all of them.  ws[c], dir[c], jump[c]: component c's solve buffers (null: the
// operator's own), Dirichlet data and interface jumps (null: zero).
template <int NC>
static int levels_multi(const hps_op *op, const Workspace *const *ws, const double *const *dir,
                        const double *const *jump, hipStream_t st, int fam_up, int fam_dn) {
    if (op->composed) return pairs_multi<NC>(op, ws, dir, jump, st, fam_up, fam_dn);
    const size_t lim = sys_lds_limit();
    auto comp_args = [&](int l, bool up, int c) {
        LevelArgs a = level_args(op, l, false, up);
        use_workspace(op, l, up, ws[c], a);
        a.dir = dir ? dir[c] : nullptr;
        a.r3 = jump ? jump[c] : nullptr;
        return a;
    };
    // the fused root only while two workgroups fit on a compute unit: above that the
    // separate up and down root launches are faster (measured at 64x64 leaves, p = 16)
    const bool rootf = root_fusable(op, false) && sys_root_lds(op, NC) <= std::min<size_t>(lim, 65536);
    {
        ProfScope ps_(&op->prof, fam_up, st);
        for (int l = op->L - 1; l >= (rootf ? 1 : 0); --l) TRY(level_multi_launch<NC>(op, l, true, ws, dir, jump, lim, st));
    }
    ProfScope ps_(&op->prof, fam_dn, st);
    if (op->L == 0) {
        for (int c = 0; c < NC; ++c) {
            hipLaunchKernelGGL(k_root_leaf_ub, dim3(1), dim3(NT), 0, st, dir ? dir[c] : nullptr,
                               (const int *)op->root_map, ws[c] ? ws[c]->ub_leaf : op->ub_leaf, 4 * op->q);
            HPS_LAUNCHED();
        }
        return HPS_OK;
    }
    if (rootf) {
        LevelSysArgsN<NC> U, Dn;
        for (int c = 0; c < NC; ++c) {
            U.c[c] = comp_args(0, true, c);
            Dn.c[c] = comp_args(0, false, c);
        }
        hipLaunchKernelGGL(k_root_sys<NC>, dim3(op->lv[0].xu64.ntile), dim3(NT), sys_root_lds(op, NC), st, U, Dn);
        HPS_LAUNCHED();
    }
    for (int l = rootf ? 1 : 0; l < op->L; ++l) TRY(level_multi_launch<NC>(op, l, false, ws, dir, jump, lim, st));
    return HPS_OK;
}

int launch_levels_sys(const hps_op *op, const Workspace *const ws[2], const double *const dir[2], hipStream_t st) {
    return levels_multi<2>(op, ws, dir, nullptr, st, KF_LEVEL2_UP64, KF_LEVEL2_DOWN64);
}

int launch_levels_multi(const hps_op *op, int nc, const Workspace *const *ws, const double *const *dir,
                        const double *const *jump, hipStream_t st) {
    switch (nc) {
        case 2: return levels_multi<2>(op, ws, dir, jump, st, KF_LEVEL_UP64, KF_LEVEL_DOWN64);
        case 3: return levels_multi<3>(op, ws, dir, jump, st, KF_LEVEL_UP64, KF_LEVEL_DOWN64);
        case 4: return levels_multi<4>(op, ws, dir, jump, st, KF_LEVEL_UP64, KF_LEVEL_DOWN64);
        default: break;
    }
    hps_set_error("internal: %d right-hand sides per level sweep", nc);
    return HPS_EINVAL;
}

// ---- argument records and launches for several operators at once (FP64) ----
size_t level_record_size() { return sizeof(LevelArgs); }

static void use_workspace(const hps_op *op, int l, bool up, const Workspace *ws, LevelArgs &a) {
    if (!ws) return;
    const bool child_leaf = (l == op->L - 1);
    a.hc = child_leaf ? ws->h_leaf : ws->lv[l + 1].h;
    a.ubc = child_leaf ? ws->ub_leaf : ws->lv[l + 1].ub;
    a.h = ws->lv[l].h;
    a.ub = ws->lv[l].ub;
    a.w3 = ws->lv[l].w3;
    a.part = ws->lv[l].part;
    a.cnt = up ? ws->lv[l].cnt_up : ws->lv[l].cnt_dn;
}

void level_record(const hps_op *op, int l, bool up, const double *dir, void *dst, int *blocks, size_t *lds,
                  const Workspace *ws, bool fp32, const double *r3) {
    LevelArgs a = level_args(op, l, fp32, up);
    use_workspace(op, l, up, ws, a);
    a.dir = dir;
    a.r3 = r3;
    *reinterpret_cast<LevelArgs *>(dst) = a;
    *blocks = op->lv[l].nodes * a.pn.ntile * a.pn.kch;
    *lds = level_lds(up ? (fp32 ? op->lv[l].xu32 : op->lv[l].xu64) : (fp32 ? op->lv[l].s32 : op->lv[l].s64));
}

bool root_fused64(const hps_op *op) { return root_fusable(op, false); }
bool root_fused(const hps_op *op, bool fp32) { return root_fusable(op, fp32); }

size_t pair_record_size() { return sizeof(PairArgs); }

int pair_lowest(const hps_op *op) { return lowest_pair(op); }

void pair_record(const hps_op *op, int l, int mode, const double *dir, void *dst, int *blocks, size_t *lds,
                 const Workspace *ws, bool fp32, const double *r3) {
    *reinterpret_cast<PairArgs *>(dst) = pair_args(op, l, mode, r3, dir, ws, fp32);
    const PairOps &P = op->pairs[l / 2];
    const Panel &pn = mode == PAIR_UP ? (fp32 ? P.up32 : P.up) : (fp32 ? P.dn32 : P.dn);
    *blocks = (int)(op->lv[l].nodes * pn.ntile);
    *lds = level_lds(pn);
}

int launch_pair_group(const void *args, const int *base, int n, int total, size_t lds, int mode, hipStream_t st,
                      bool fp32) {
    if (total <= 0) return HPS_OK;
    const PairArgs *a = reinterpret_cast<const PairArgs *>(args);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(total), dim3(NT), lds, st, a, base, n); };
    if (fp32) {
        if (mode == PAIR_UP) go(k_pair_group<float, PAIR_UP>);
        else if (mode == PAIR_DOWN) go(k_pair_group<float, PAIR_DOWN>);
        else go(k_pair_group<float, PAIR_TOP>);
    } else {
        if (mode == PAIR_UP) go(k_pair_group<double, PAIR_UP>);
        else if (mode == PAIR_DOWN) go(k_pair_group<double, PAIR_DOWN>);
        else go(k_pair_group<double, PAIR_TOP>);
    }
    HPS_LAUNCHED();
    return HPS_OK;
}

void root_records(const hps_op *op, const double *dir, void *up_dst, void *dn_dst, int *blocks, size_t *lds,
                  const Workspace *ws, bool fp32, const double *r3) {
    LevelArgs up = level_args(op, 0, fp32, true), dn = level_args(op, 0, fp32, false);
    use_workspace(op, 0, true, ws, up);
    use_workspace(op, 0, false, ws, dn);
    up.r3 = r3;
    dn.dir = dir;
    *reinterpret_cast<LevelArgs *>(up_dst) = up;
    *reinterpret_cast<LevelArgs *>(dn_dst) = dn;
    const Panel &x = fp32 ? op->lv[0].xu32 : op->lv[0].xu64, &sp = fp32 ? op->lv[0].s32 : op->lv[0].s64;
    *blocks = x.ntile;
    *lds = level_lds(x) + level_lds(sp) + 32;
}

size_t eval_record_size() { return sizeof(EvalArgs); }
size_t jump_record_size() { return sizeof(JumpArgs); }

void residual_records(const hps_op *op, const double *u, const double *rhs, double *r_int, double *r3, double *flux,
                      void *eval_dst, void *jump_dst, int *leaves, int *iface) {
    EvalArgs a{};
    a.geo = geo_of(op);
    a.u = u;
    a.D = op->D;
    a.D2 = op->D2;
    a.coef = op->coef;
    a.rhs = rhs;
    a.gamma_dt = op->gamma_dt;
    a.r_int = r_int;
    a.flux = flux;
    *reinterpret_cast<EvalArgs *>(eval_dst) = a;
    *reinterpret_cast<JumpArgs *>(jump_dst) = JumpArgs{geo_of(op), flux, nullptr, 1.0, r3, op->n_iface};
    *leaves = op->nleaves;
    *iface = (int)op->n_iface;
}

int launch_residual_group(const void *evals, const int *ebase, const void *jumps, const int *jbase, int n,
                          int total_leaves, int total_iface, hipStream_t st) {
    if (total_leaves > 0) {
        hipLaunchKernelGGL(k_eval_group, dim3(total_leaves), dim3(NT), 0, st, reinterpret_cast<const EvalArgs *>(evals),
                           ebase, n);
        HPS_LAUNCHED();
    }
    if (total_iface > 0) {
        hipLaunchKernelGGL(k_jump_group, dim3(nblk(total_iface)), dim3(NT), 0, st,
                           reinterpret_cast<const JumpArgs *>(jumps), jbase, n);
        HPS_LAUNCHED();
    }
    return HPS_OK;
}

int launch_norm_fold(const double *part, int leaves, double *out, hipStream_t st) {
    NormFold f{part, reinterpret_cast<unsigned long long *>(out), leaves};
    hipLaunchKernelGGL(k_norm_fold, dim3(1), dim3(NT), 0, st, f);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_norm_fold_group(const NormFold *folds, int n, hipStream_t st) {
    if (n <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_norm_fold_group, dim3(n), dim3(NT), 0, st, folds);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_memop_group(const MemOp *ops, const int64_t *base, int n, int64_t total, hipStream_t st) {
    if (total <= 0) return HPS_OK;
    const unsigned gx = (unsigned)std::min<int64_t>(nblk(total), 4096);
    hipLaunchKernelGGL(k_memop_group, dim3(gx), dim3(NT), 0, st, ops, base, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

size_t line_record_size() { return sizeof(LineArgs); }

void line_record(const hps_op *op, double *u, void *dst, int *systems, const Workspace *ws) {
    LineArgs la{};
    la.geo = geo_of(op);
    la.u = u;
    la.fpart = ws ? ws->flux : op->ir_flux;
    la.D = op->D;
    la.cp = op->tri_cp;
    la.inv_den = op->tri_cp + op->tri_stride;
    *reinterpret_cast<LineArgs *>(dst) = la;
    *systems = op->grid.n2 * op->q + op->grid.n1 * op->q;
}

size_t scatter_record_size() { return sizeof(ScatterTask); }

void scatter_record(const hps_op *op, double *u, void *dst, int *count) {
    *reinterpret_cast<ScatterTask *>(dst) = ScatterTask{op->bnd_glob, u};
    *count = (int)op->n_bdry;
}

int launch_level_group(const void *args, const int *base, int n, int total, size_t lds, bool up, hipStream_t st,
                       bool fp32) {
    if (total <= 0) return HPS_OK;
    const LevelArgs *a = reinterpret_cast<const LevelArgs *>(args);
    if (fp32) {
        if (up) hipLaunchKernelGGL((k_level_group<float, true>), dim3(total), dim3(NT), lds, st, a, base, n);
        else hipLaunchKernelGGL((k_level_group<float, false>), dim3(total), dim3(NT), lds, st, a, base, n);
    } else {
        if (up) hipLaunchKernelGGL((k_level_group<double, true>), dim3(total), dim3(NT), lds, st, a, base, n);
        else hipLaunchKernelGGL((k_level_group<double, false>), dim3(total), dim3(NT), lds, st, a, base, n);
    }
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_root_group(const void *ups, const void *dns, const int *base, int n, int total, size_t lds,
                      hipStream_t st, bool fp32) {
    if (total <= 0) return HPS_OK;
    const LevelArgs *u = reinterpret_cast<const LevelArgs *>(ups), *d = reinterpret_cast<const LevelArgs *>(dns);
    if (fp32) hipLaunchKernelGGL(k_root_group<float>, dim3(total), dim3(NT), lds, st, u, d, base, n);
    else hipLaunchKernelGGL(k_root_group<double>, dim3(total), dim3(NT), lds, st, u, d, base, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_lines_group(const void *args, const int *base, int n, int total, hipStream_t st) {
    if (total <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_lines_group, dim3(nblk(total, 64)), dim3(64), 0, st, reinterpret_cast<const LineArgs *>(args),
                       base, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_zero_boundary_group(const void *args, const int *base, int n, int total, hipStream_t st) {
    if (total <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_zero_boundary_group, dim3(nblk(total)), dim3(NT), 0, st,
                       reinterpret_cast<const ScatterTask *>(args), base, n);
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
                           (const double *)op->ir_flux, jump, 1.0, r3, op->n_iface);
        HPS_LAUNCHED();
    }
    return HPS_OK;
}

int launch_interface_lines(const hps_op *op, double *u, const double *f_end, hipStream_t st,
                           const double *jump, const double *fpart) {
    ProfScope ps_(&op->prof, KF_LINES, st);
    LineArgs la{};
    la.geo = geo_of(op);
    la.u = u;
    la.fpart = fpart ? fpart : op->ir_flux;
    la.D = op->D;
    la.cp = op->tri_cp;
    la.inv_den = op->tri_cp + op->tri_stride;
    la.jump = jump;
    const int nsys = op->grid.n2 * op->q + op->grid.n1 * op->q;
    const int nmax = std::max(op->grid.n1, op->grid.n2);
    const size_t lds = ((size_t)nmax * LINES + 2 * (size_t)nmax) * sizeof(double);
    if (lds <= sys_lds_limit()) {   // the boundary scatter in the same launch
        la.f = f_end;
        la.ends = op->line_ends;
        la.bnd_glob = op->bnd_glob;
        la.nb = op->n_bdry;
        hipLaunchKernelGGL(k_interface_lines_lds, dim3(nblk(nsys, LINES)), dim3(LINE_NT), lds, st, la, nmax);
    } else {   // lines too long to stage in LDS: one thread per line, inputs read from memory
        TRY(launch_scatter_boundary(op, f_end, u, st));
        hipLaunchKernelGGL(k_interface_lines, dim3(nblk(nsys, 64)), dim3(64), 0, st, la);
    }
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_scatter_boundary(const hps_op *op, const double *f, double *u, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_boundary, dim3(nblk(op->n_bdry)), dim3(NT), 0, st, f,
                       (const int *)op->bnd_glob, u, op->n_bdry);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_set_values(double *dst, const double *vals, int n, hipStream_t st) {
    if (n <= 0) return HPS_OK;
    if (n > 8) {
        hps_set_error("internal: at most 8 values per launch_set_values");
        return HPS_EINVAL;
    }
    Values8 v{};
    for (int i = 0; i < n; ++i) v.v[i] = vals[i];
    hipLaunchKernelGGL(k_set_values, dim3(1), dim3(64), 0, st, dst, v, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

// out = g(sum_k c_k v_k + qs q) over n entries (g applied when g.kind != 0); qs is the
// device scalar *q_scale_ptr when given, else 1.  out may alias one of the inputs.
struct LinComb {
    const double *v[kMaxLinComb];
    double c[kMaxLinComb];
    int nv;
    const double *q;
    const double *q_scale_ptr;
    GPoly g;
    double *out;
    int64_t n;
};

__global__ void k_lincomb(LinComb a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double s = 0.0;
    for (int k = 0; k < a.nv; ++k) s = fma(a.c[k], a.v[k][i], s);
    if (a.q) s = fma(a.q_scale_ptr ? *a.q_scale_ptr : 1.0, a.q[i], s);
    if (a.g.kind) s = gpoly(a.g, s);
    a.out[i] = s;
}

int launch_lincomb(const double *const *v, const double *c, int nv, const double *q, const double *q_scale_ptr,
                   const GPoly *g, double *out, int64_t n, hipStream_t st) {
    if (n <= 0) return HPS_OK;
    if (nv > kMaxLinComb) {
        hps_set_error("internal: %d terms exceed the %d a combination takes", nv, kMaxLinComb);
        return HPS_EINVAL;
    }
    LinComb a{};
    for (int k = 0; k < nv; ++k) {
        a.v[k] = v[k];
        a.c[k] = c[k];
    }
    a.nv = nv;
    a.q = q;
    a.q_scale_ptr = q_scale_ptr;
    if (g) a.g = *g;
    a.out = out;
    a.n = n;
    hipLaunchKernelGGL(k_lincomb, dim3(nblk(n)), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

// L v at interior nodes (into Lu, if given) and, when `flux` is set, the coordinate-
// direction fluxes of v on every leaf edge into op->ir_flux, from a canonical vector v.
int launch_eval(const hps_op *op, const double *v, double *Lu, bool flux, hipStream_t st) {
    EvalArgs a{};
    a.geo = geo_of(op);
    a.u = v;
    a.D = op->D;
    a.D2 = op->D2;
    a.coef = op->coef;
    a.Lu = Lu;
    a.flux = flux ? op->ir_flux : nullptr;
    hipLaunchKernelGGL(k_eval, dim3(op->nleaves), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

// r3 = -scale (flux_alpha - flux_beta) per interface node, from the fluxes in op->ir_flux
int launch_flux_jump(const hps_op *op, double scale, double *r3, hipStream_t st) {
    if (op->n_iface <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_jump, dim3(nblk(op->n_iface)), dim3(NT), 0, st, geo_of(op), (const double *)op->ir_flux,
                       (const double *)nullptr, scale, r3, op->n_iface);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_zero(double *p, int64_t n, hipStream_t st) {
    if (n <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(NT), 0, st, p, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_copy(double *dst, const double *src, int64_t n, hipStream_t st) {
    if (n <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(NT), 0, st, dst, src, n);
    HPS_LAUNCHED();
    return HPS_OK;
}

}  // namespace hps
