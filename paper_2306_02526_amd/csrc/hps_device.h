// Device-side helpers shared by the solve and build kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hps_internal.h"

namespace hps {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

template <typename T> struct V16;
template <> struct V16<double> { using type = dvec2; };
template <> struct V16<float> { using type = fvec4; };

__device__ __forceinline__ void vfma(double *acc, const dvec2 &v, double x) {
    acc[0] = fma(v.x, x, acc[0]);
    acc[1] = fma(v.y, x, acc[1]);
}
__device__ __forceinline__ void vfma(float *acc, const fvec4 &v, float x) {
    acc[0] = fmaf(v.x, x, acc[0]);
    acc[1] = fmaf(v.y, x, acc[1]);
    acc[2] = fmaf(v.z, x, acc[2]);
    acc[3] = fmaf(v.w, x, acc[3]);
}

struct PanelView {
    const void *data;
    int rp, G, S, ntile, kch;
    int64_t tile_elems, node_elems;
};

inline PanelView view(const Panel &p) {
    // a shared panel has one block that every node reads
    return PanelView{p.data, p.rp, p.G, p.S, p.ntile, p.kch, p.tile_elems, p.shared ? 0 : p.node_elems};
}

// Streaming product of one (tile, chunk) block of a Panel with an LDS vector.
// start(): issue the first PF 16-byte loads of this lane (they do not depend on the
// input vector, so callers start them before gathering it); finish(): consume them and
// stream the rest with UNR loads in flight, then store the lane's partial sums.
// Operators read once per sweep use nontemporal loads; a shared panel (one copy read by
// every node, `cached`) uses ordinary loads so that the copy stays in the caches.
template <typename T, int PF, int UNR>
struct PanelStream {
    using V = typename V16<T>::type;
    static constexpr int VW = 16 / sizeof(T);
    const V *p;
    int act, S, G, g, r;
    bool on, nt;
    V pre[PF];

    template <bool NTL>
    static __device__ __forceinline__ V ld(const V *q) {
        if constexpr (NTL) return __builtin_nontemporal_load(q);
        else return *q;
    }

    __device__ __forceinline__ void start(const T *blk, int rp, int G_, int S_, bool cached = false) {
        const int t = threadIdx.x;
        act = rp * G_;
        S = S_;
        G = G_;
        on = t < act;
        nt = !cached;
        g = on ? t / rp : 0;
        r = on ? t - g * rp : 0;
        p = reinterpret_cast<const V *>(blk) + t;
        if (on) {
            if (nt) {
#pragma unroll
                for (int u = 0; u < PF; ++u)
                    if (u < S) pre[u] = ld<true>(p + (size_t)u * act);
            } else {
#pragma unroll
                for (int u = 0; u < PF; ++u)
                    if (u < S) pre[u] = ld<false>(p + (size_t)u * act);
            }
        }
    }

    // NC input vectors at once (vector c at xs + c*xstride, its partial sums to
    // part + c*pstride): every operator load feeds NC products.
    template <bool NTL, int NC>
    __device__ __forceinline__ void run(const T *__restrict__ xs, int xstride, T *__restrict__ part, int pstride) {
        T acc[NC][VW];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int v = 0; v < VW; ++v) acc[c][v] = T(0);
#pragma unroll
        for (int u = 0; u < PF; ++u)
            if (u < S)
#pragma unroll
                for (int c = 0; c < NC; ++c) vfma(acc[c], pre[u], xs[c * xstride + u * G + g]);
        int s = PF;
        for (; s + UNR <= S; s += UNR) {
            V vv[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) vv[u] = ld<NTL>(p + (size_t)(s + u) * act);
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int c = 0; c < NC; ++c) vfma(acc[c], vv[u], xs[c * xstride + (s + u) * G + g]);
        }
        for (; s < S; ++s) {
            const V w = ld<NTL>(p + (size_t)s * act);
#pragma unroll
            for (int c = 0; c < NC; ++c) vfma(acc[c], w, xs[c * xstride + s * G + g]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            T *dst = part + c * pstride + g * (act / G * VW) + r * VW;
#pragma unroll
            for (int v = 0; v < VW; ++v) dst[v] = acc[c][v];
        }
    }

    __device__ __forceinline__ void finish(const T *__restrict__ xs, T *__restrict__ part) {
        if (!on) return;
        if (nt) run<true, 1>(xs, 0, part, 0);
        else run<false, 1>(xs, 0, part, 0);
    }

    template <int NC>
    __device__ __forceinline__ void finish_n(const T *__restrict__ xs, int xstride, T *__restrict__ part,
                                             int pstride) {
        if (!on) return;
        if (nt) run<true, NC>(xs, xstride, part, pstride);
        else run<false, NC>(xs, xstride, part, pstride);
    }
};

template <typename T>
__device__ __forceinline__ double panel_sum(const T *__restrict__ part, int rp, int G, int idx) {
    constexpr int VW = 16 / sizeof(T);
    T s = T(0);
    for (int g = 0; g < G; ++g) s += part[g * (rp * VW) + idx];
    return (double)s;
}

// LDS carve-up helper for dynamic shared memory
struct Carve {
    unsigned char *base;
    size_t off = 0;
    template <typename T>
    __device__ __forceinline__ T *take(size_t n) {
        off = (off + 15) & ~size_t(15);
        T *ptr = reinterpret_cast<T *>(base + off);
        off += n * sizeof(T);
        return ptr;
    }
};

inline size_t carve_bytes(std::initializer_list<size_t> sizes) {
    size_t off = 0;
    for (size_t s : sizes) off = ((off + 15) & ~size_t(15)) + s;
    return off;
}

struct LeafGeo {
    int n1, n2, q, p;
    int64_t n_int, n_vert;
};

inline LeafGeo geo_of(const hps_op *op) {
    return LeafGeo{op->grid.n1, op->grid.n2, op->q, op->p, op->n_int, op->n_vert};
}

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

// L u = cxx u_xx + cyy u_yy + cx u_x + cy u_y + c0 u at one node (eq. 3 for L, c12 = 0), the
// coefficients c[0..4] in that order, as explicit fused multiply-adds: every kernel that
// evaluates L u (stage vectors, refinement residuals) rounds it the same way
__device__ __forceinline__ double apply_L_point(const double *c, double uxx, double uyy, double ux, double uy,
                                                double u) {
    return fma(c[4], u, fma(c[3], uy, fma(c[2], ux, fma(c[1], uyy, c[0] * uxx))));
}

// Row stride of a p x p differentiation matrix kept in LDS for tile derivatives: lanes of
// a wave read one row each (one per interior column of the tile), and with stride p + 1
// those rows fall in different banks instead of all in one
__host__ __device__ constexpr int dmat_ld(int p) { return p + 1; }

__device__ __forceinline__ void load_dmat_ld(const double *src, double *dst, int p) {
    const int ld = dmat_ld(p);
    for (int k = threadIdx.x; k < p * p; k += blockDim.x) {
        const int r = k / p;
        dst[r * ld + (k - r * p)] = src[k];
    }
}

static inline unsigned nblk(int64_t n, int t = NT) { return (unsigned)((n + t - 1) / t); }

}  // namespace hps
