// HIP kernels of the HPS build on gfx950: leaf operators (Sec. 2.1, eqs. 5-6), batched
// Gauss-Jordan inversion, the merge gather and the FP64 MFMA GEMM for the merge formulas
// after eqs. (7)-(8), and the packing of the stored operators into streaming order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>

#include "hps_device.h"

namespace hps {

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

// ---- complex operators (Sec. 5.5): real embeddings --------------------------------------
// A complex matrix M = Mr + i Mi acts on (Re z, Im z) as [[Mr, -Mi], [Mi, Mr]].  The
// coefficient planes of a complex operator hold the 5 real parts, then the 5 imaginary
// parts; A = I - gdt L has real part I - gdt L_re and imaginary part -gdt L_im.

// entry (r, c) of the interior block of L's coefficient plane set `co` (identity excluded)
__device__ __forceinline__ double leaf_L_entry(const double *co, int64_t n_int, int64_t gi, const double *D,
                                               const double *D2, int p, int a1, int b1, int a2, int b2) {
    double v = 0.0;
    if (b1 == b2) v += co[gi] * D2[a1 * p + a2] + co[2 * n_int + gi] * D[a1 * p + a2];
    if (a1 == a2) v += co[n_int + gi] * D2[b1 * p + b2] + co[3 * n_int + gi] * D[b1 * p + b2];
    if (a1 == a2 && b1 == b2) v += co[4 * n_int + gi];
    return v;
}

// embedded A_ii (2 q2 x 2 q2, column-major) on every leaf
__global__ __launch_bounds__(NT) void k_leaf_assemble_cx(BuildLeafArgs a, double *W) {
    __shared__ double D[PMAX * PMAX], D2[PMAX * PMAX];
    const int leaf = blockIdx.y;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, n = 2 * q2;
    load_dmat(a.D, D, p * p);
    load_dmat(a.D2, D2, p * p);
    __syncthreads();
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int64_t n_int = a.geo.n_int;
    const int64_t tot = (int64_t)n * n;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        const int R = (int)(idx % n), Cc = (int)(idx / n);
        const int cr = R / q2, r = R % q2, cc = Cc / q2, c = Cc % q2;
        const int a1 = r % q + 1, b1 = r / q + 1, a2 = c % q + 1, b2 = c / q + 1;
        const int64_t gi = base + r;
        double v;
        if (cr == cc) {   // real part: I - gdt L_re
            v = -a.gamma_dt * leaf_L_entry(a.coef, n_int, gi, D, D2, p, a1, b1, a2, b2) + (r == c ? 1.0 : 0.0);
        } else {          // imaginary part -gdt L_im, with the sign of its block
            const double im = -a.gamma_dt * leaf_L_entry(a.coef + 5 * n_int, n_int, gi, D, D2, p, a1, b1, a2, b2);
            v = (cr == 1) ? im : -im;
        }
        W[(int64_t)leaf * tot + idx] = v;
    }
}

// embedded S_leaf = -A_ii^{-1} A_ib (2 q2 x 8 q): boundary column (cc, e, m)
__global__ __launch_bounds__(NT) void k_leaf_S_cx(BuildLeafArgs a, const double *ainv, double *S) {
    __shared__ double D[PMAX * PMAX], D2[PMAX * PMAX];
    const int leaf = blockIdx.y;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q, n = 2 * q2;
    load_dmat(a.D, D, p * p);
    load_dmat(a.D2, D2, p * p);
    __syncthreads();
    const int li = a.leaf_ij[2 * leaf], lj = a.leaf_ij[2 * leaf + 1];
    const int64_t base = ((int64_t)lj * a.geo.n1 + li) * q2;
    const int64_t n_int = a.geo.n_int;
    const double gdt = a.gamma_dt;
    const double *Ai = ainv + (int64_t)leaf * n * n;
    const int64_t tot = (int64_t)n * 2 * nb;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        const int R = (int)(idx % n), col2 = (int)(idx / n);
        const int cc = col2 / nb, col = col2 % nb;
        const int e = col / q, m = col % q;
        double s = 0.0;
        for (int c = 1; c <= q; ++c) {
            int rho;
            double vre, vim;   // real and imaginary part of the A_ib entry (row rho, this node)
            if (e < 2) {
                rho = m * q + (c - 1);
                const int ap = (e == 0) ? 0 : p - 1;
                const int64_t gi = base + rho;
                vre = -gdt * (a.coef[gi] * D2[c * p + ap] + a.coef[2 * n_int + gi] * D[c * p + ap]);
                vim = -gdt * (a.coef[5 * n_int + gi] * D2[c * p + ap] + a.coef[7 * n_int + gi] * D[c * p + ap]);
            } else {
                rho = (c - 1) * q + m;
                const int bp = (e == 2) ? 0 : p - 1;
                const int64_t gi = base + rho;
                vre = -gdt * (a.coef[n_int + gi] * D2[c * p + bp] + a.coef[3 * n_int + gi] * D[c * p + bp]);
                vim = -gdt * (a.coef[6 * n_int + gi] * D2[c * p + bp] + a.coef[8 * n_int + gi] * D[c * p + bp]);
            }
            // column cc of the embedded A_ib: rows of component 0 and 1
            const double top = (cc == 0) ? vre : -vim;   // block (0, cc)
            const double bot = (cc == 0) ? vim : vre;    // block (1, cc)
            s = fma(Ai[(int64_t)rho * n + R], top, s);
            s = fma(Ai[(int64_t)(q2 + rho) * n + R], bot, s);
        }
        S[(int64_t)leaf * tot + idx] = -s;
    }
}

// embedded DtN map (8 q x 8 q): the flux rows act on each component separately
__global__ __launch_bounds__(NT) void k_leaf_T_cx(BuildLeafArgs a, const double *S, double *T) {
    __shared__ double D[PMAX * PMAX];
    const int leaf = blockIdx.y;
    const int q = a.geo.q, p = a.geo.p, q2 = q * q, nb = 4 * q, n = 2 * q2, nbl = 2 * nb;
    load_dmat(a.D, D, p * p);
    __syncthreads();
    const double *Sl = S + (int64_t)leaf * n * nbl;
    const int64_t tot = (int64_t)nbl * nbl;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        const int row2 = (int)(idx % nbl), col = (int)(idx / nbl);
        const int cr = row2 / nb, row = row2 % nb;
        const int e = row / q, m = row % q;
        const double *dr = D + ((e == 0 || e == 2) ? 0 : (p - 1) * p);
        double v = 0.0;
        for (int c = 1; c <= q; ++c) {
            const int rho = (e < 2) ? m * q + (c - 1) : (c - 1) * q + m;
            v = fma(dr[c], Sl[(int64_t)col * n + cr * q2 + rho], v);
        }
        const int lo = cr * nb + ((e < 2) ? 0 * q + m : 2 * q + m);
        const int hi = cr * nb + ((e < 2) ? 1 * q + m : 3 * q + m);
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
    int64_t cstride;   // elements between children's T in Tc (0: every node's children are T[0])
};

__global__ __launch_bounds__(NT) void k_merge_gather(MergeArgs a) {
    const int node = blockIdx.y;
    const double *Ta = a.Tc + (int64_t)(2 * node) * a.cstride;
    const double *Tb = a.Tc + (int64_t)(2 * node + 1) * a.cstride;
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
        if ((int)threadIdx.x < off) {
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

// Update of step k and pivot of step k + 1 in one launch: the batch is read from Ws and
// written to Wd (two copies in turn), so the first nb workgroups (`npiv`, one per matrix;
// none after the last step) can compute step k's result for column k + 1 and for the new
// pivot row themselves, with the same operations as the update, while the other
// workgroups write every element.  Step k's column and row come from cbk / rbk, step
// k + 1's go to cbn / rbn.  Bitwise the same as k_gj_update followed by k_gj_pivot.
__global__ __launch_bounds__(NT) void k_gj_step(const double *Ws, double *Wd, int n, int nb, int k, int npiv,
                                                unsigned char *used, int *order, const double *cbk,
                                                const double *rbk, double *cbn, double *rbn, int *sing) {
    const int64_t nn = (int64_t)n * n;
    if ((int)blockIdx.x >= npiv) {
        const int64_t idx = (int64_t)(blockIdx.x - npiv) * NT + threadIdx.x;
        if (idx >= nn * nb) return;
        const int b = (int)(idx / nn);
        const int64_t rem = idx - b * nn;
        const int j = (int)(rem / n), i = (int)(rem % n);
        const int pr = order[(int64_t)b * n + k];
        const double *cb = cbk + (int64_t)b * n;
        const double *rb = rbk + (int64_t)b * n;
        if (i == pr) Wd[idx] = rb[j];
        else if (j == k) Wd[idx] = -cb[i] * rb[k];
        else Wd[idx] = fma(-cb[i], rb[j], Ws[idx]);
        return;
    }
    __shared__ double bv[NT];
    __shared__ int bi[NT];
    const int b = blockIdx.x, k1 = k + 1;
    const double *Wb = Ws + (int64_t)b * nn;
    const double *cb = cbk + (int64_t)b * n;
    const double *rb = rbk + (int64_t)b * n;
    double *cn = cbn + (int64_t)b * n;
    unsigned char *ub = used + (int64_t)b * n;
    const int pk = order[(int64_t)b * n + k];
    // column k + 1 after step k (never column k itself)
    double best = -1.0;
    int besti = n;
    for (int i = threadIdx.x; i < n; i += NT) {
        const double v = (i == pk) ? rb[k1] : fma(-cb[i], rb[k1], Wb[(int64_t)k1 * n + i]);
        cn[i] = v;
        if (!ub[i]) {
            const double a = fabs(v);
            if (a > best || (a == best && i < besti)) {
                best = a;
                besti = i;
            }
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = besti;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
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
    if (pr < n) piv = cn[pr];
    if (pr >= n || piv == 0.0 || !isfinite(piv)) {
        if (threadIdx.x == 0) atomicExch(sing, 1);
        if (pr >= n) pr = 0;
        piv = 1.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ub[pr] = 1;
        order[(int64_t)b * n + k1] = pr;
    }
    const double ip = 1.0 / piv;
    double *rn = rbn + (int64_t)b * n;
    // the new pivot row after step k, scaled
    for (int j = threadIdx.x; j < n; j += NT) {
        double v;
        if (pr == pk) v = rb[j];
        else if (j == k) v = -cb[pr] * rb[k];
        else v = fma(-cb[pr], rb[j], Wb[(int64_t)j * n + pr]);
        rn[j] = (j == k1) ? ip : v * ip;
    }
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

// ---- the same inversion with one matrix per workgroup, held in registers ---------------
// A GJ_TR x GJ_TC grid of threads holds the n x n matrix: thread (r, c) owns rows
// r + GJ_TR a (a < RA) and columns c + GJ_TC b (b < CB), n <= GJ_TR RA and n <= GJ_TC CB, so
// every step touches the matrix in registers instead of streaming the whole batch through
// memory twice per step (512 threads: up to 256 registers per lane, 13 x 7 doubles each
// at n = 196).  Each step performs exactly the operations of k_gj_pivot / k_gj_update (same
// pivot rule, same products and fused multiply-adds), so the result is bitwise that of the
// batched kernels; the unpermutation is done on the way out.
//
// Two barriers per step.  Every wave finds the pivot itself from the column in LDS (the
// same deterministic search, so all waves agree; each keeps the used-row flags of its
// lanes' rows in a register), the owners of the pivot row publish it scaled, and after the
// barrier every element takes one fused multiply-add, the pivot row and column k being
// overwritten afterwards; the owners of column k + 1 publish it into the other half of a
// double-buffered column in the same phase.
constexpr int GJ_TR = 16, GJ_TC = 32;   // thread grid: rows x columns
constexpr int GJ_NT = GJ_TR * GJ_TC;
constexpr int GJ_MAXN = 256;            // rows a wave's pivot search covers (4 per lane)

static size_t gj_reg_lds(int n) { return (size_t)n * (3 * sizeof(double) + 2 * sizeof(int)); }

template <int RA, int CB>
__global__ __launch_bounds__(GJ_NT) void k_gj_reg(const double *W, double *out, int n, int *sing) {
    static_assert(GJ_TR * RA <= GJ_MAXN, "the pivot search covers at most GJ_MAXN rows");
    extern __shared__ __align__(16) unsigned char gsm[];
    double *colbuf = reinterpret_cast<double *>(gsm);        // [2][n] column k, by step parity
    double *rowbuf = colbuf + 2 * n;                          // [n] scaled pivot row
    int *order = reinterpret_cast<int *>(rowbuf + n);         // [n] pivot row of step k
    int *pinv = order + n;                                    // [n] step of pivot row i
    const int t = threadIdx.x, b = blockIdx.x, lane = t & 63;
    const int r = t % GJ_TR, c = t / GJ_TR;
    const int64_t nn = (int64_t)n * n;
    const double *Wb = W + b * nn;
    double w[RA][CB];   // w[a][bb] = W[r + GJ_TR a][c + GJ_TC bb]
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int bb = 0; bb < CB; ++bb) {
            const int i = r + GJ_TR * a, j = c + GJ_TC * bb;
            w[a][bb] = (i < n && j < n) ? Wb[(int64_t)j * n + i] : 0.0;
        }
    for (int i = t; i < n; i += GJ_NT) {
        order[i] = i;   // complete permutations even if a singular step repeats a row
        pinv[i] = i;
    }
    if (c == 0)
#pragma unroll
        for (int a = 0; a < RA; ++a) {
            const int i = r + GJ_TR * a;
            if (i < n) colbuf[i] = w[a][0];
        }
    unsigned used = 0;   // bit m: row lane + 64 m is a pivot row already
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double *col = colbuf + (k & 1) * n;
        // unused row with the largest |W[i][k]|, ties to the smallest i (every wave)
        double best = -1.0;
        int besti = n;
#pragma unroll
        for (int m = 0; m < GJ_MAXN / 64; ++m) {
            const int i = lane + 64 * m;
            if (i < n && !((used >> m) & 1u)) {
                const double v = fabs(col[i]);
                if (v > best || (v == best && i < besti)) {
                    best = v;
                    besti = i;
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double v2 = __shfl_xor(best, off);
            const int i2 = __shfl_xor(besti, off);
            if (v2 > best || (v2 == best && i2 < besti)) {
                best = v2;
                besti = i2;
            }
        }
        int pr = besti;
        double piv = pr < n ? col[pr] : 0.0;
        if (pr >= n || piv == 0.0 || !isfinite(piv)) {
            if (t == 0) atomicExch(sing, 1);
            if (pr >= n) pr = 0;
            piv = 1.0;
        }
        const double ip = 1.0 / piv;
        if (lane == (pr & 63)) used |= 1u << (pr >> 6);
        if (t == 0) {
            order[k] = pr;
            pinv[pr] = k;
        }
        // the pivot row, scaled (thread row r == pr % GJ_TR holds it)
        if (r == pr % GJ_TR) {
            const int ap = pr / GJ_TR;
#pragma unroll
            for (int a = 0; a < RA; ++a)
                if (a == ap)
#pragma unroll
                    for (int bb = 0; bb < CB; ++bb) {
                        const int j = c + GJ_TC * bb;
                        if (j < n) rowbuf[j] = (j == k) ? ip : w[a][bb] * ip;
                    }
        }
        __syncthreads();
        double cb[RA], rb[CB];
#pragma unroll
        for (int a = 0; a < RA; ++a) {
            const int i = r + GJ_TR * a;
            cb[a] = i < n ? col[i] : 0.0;
        }
#pragma unroll
        for (int bb = 0; bb < CB; ++bb) {
            const int j = c + GJ_TC * bb;
            rb[bb] = j < n ? rowbuf[j] : 0.0;
        }
        const double rbk = rowbuf[k];
        // padding rows and columns (cb or rb zero) keep zeros and are never read
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int bb = 0; bb < CB; ++bb) w[a][bb] = fma(-cb[a], rb[bb], w[a][bb]);
        if (c == k % GJ_TC) {   // column k of the rows other than the pivot row
            const int bk = k / GJ_TC;
#pragma unroll
            for (int bb = 0; bb < CB; ++bb)
                if (bb == bk)
#pragma unroll
                    for (int a = 0; a < RA; ++a) w[a][bb] = -cb[a] * rbk;
        }
        if (r == pr % GJ_TR) {   // the pivot row
            const int ap = pr / GJ_TR;
#pragma unroll
            for (int a = 0; a < RA; ++a)
                if (a == ap)
#pragma unroll
                    for (int bb = 0; bb < CB; ++bb) w[a][bb] = rb[bb];
        }
        // column k + 1 for the next step (thread column c == (k + 1) % GJ_TC holds it)
        const int k1 = k + 1;
        if (k1 < n && c == k1 % GJ_TC) {
            const int bk = k1 / GJ_TC;
            double *nxt = colbuf + (k1 & 1) * n;
#pragma unroll
            for (int bb = 0; bb < CB; ++bb)
                if (bb == bk)
#pragma unroll
                    for (int a = 0; a < RA; ++a) {
                        const int i = r + GJ_TR * a;
                        if (i < n) nxt[i] = w[a][bb];
                    }
        }
        __syncthreads();
    }
    // inv(A)[k][order[j]] = W[order[k]][j]: element (i, j) goes to row pinv[i], column order[j]
    double *ob = out + b * nn;
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int bb = 0; bb < CB; ++bb) {
            const int i = r + GJ_TR * a, j = c + GJ_TC * bb;
            if (i < n && j < n) ob[(int64_t)order[j] * n + pinv[i]] = w[a][bb];
        }
}

// ---- batched FP64 GEMM on the matrix cores ----------------------------------------------
// C = alpha A B + beta C, column-major, 64x64 tile per workgroup, each wave a 32x32
// sub-tile of 2x2 v_mfma_f64_16x16x4 blocks; K staged through LDS 16 at a time, the next
// 16 loaded into registers while the current ones are multiplied (one barrier per step).
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
    constexpr int LA = TM * TK / NT, LB = TN * TK / NT;   // elements per thread and tile
    static_assert(NT == 256 && LA == 4 && LB == 4, "tile loads assume 256 threads");
    // two LDS buffers: the tile in use and the next one; the next tile's global loads are
    // in flight in registers while the matrix cores work on the current one
    __shared__ double As[2][TK][TM + 1];
    __shared__ double Bs[2][TK][TN + 1];
    const int bz = blockIdx.z;
    const double *A = g.A + bz * g.sA;
    const double *B = g.B + bz * g.sB;
    double *C = g.C + bz * g.sC;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    // this thread's tile elements: A rows ai, k rows ak + 4 r; B k row bk, columns bj + 16 r
    const int ai = t % TM, ak = t / TM, bk = t % TK, bj = t / TK;
    double ra[LA], rb[LB];
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int gm = m0 + ai, gk = k0 + ak + 4 * r;
            ra[r] = (gm < g.M && gk < g.K) ? A[(int64_t)gk * g.lda + gm] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const int gn = n0 + bj + 16 * r, gk = k0 + bk;
            rb[r] = (gn < g.N && gk < g.K) ? B[(int64_t)gn * g.ldb + gk] : 0.0;
        }
    };
    dvec4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = dvec4{0.0, 0.0, 0.0, 0.0};
    load(0);
    int buf = 0;
    for (int k0 = 0; k0 < g.K; k0 += TK) {
#pragma unroll
        for (int r = 0; r < LA; ++r) As[buf][ak + 4 * r][ai] = ra[r];
#pragma unroll
        for (int r = 0; r < LB; ++r) Bs[buf][bk][bj + 16 * r] = rb[r];
        __syncthreads();
        if (k0 + TK < g.K) load(k0 + TK);
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = As[buf][kk + lk][wm * 32 + x * 16 + li];
#pragma unroll
            for (int y = 0; y < 2; ++y) bv[y] = Bs[buf][kk + lk][wn * 32 + y * 16 + li];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
        }
        buf ^= 1;
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
    double scale;
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
    reinterpret_cast<T *>(a.dst)[idx] = (T)(val * a.scale);
}

// =======================================================================================
// launchers
// =======================================================================================
// leaves whose operators the build computes (one when all leaves have the same operators)
static unsigned build_leaves(const hps_op *op) { return op->build_one ? 1u : (unsigned)op->nleaves; }

static BuildLeafArgs build_leaf_args(const hps_op *op) {
    return BuildLeafArgs{geo_of(op), op->leaf_ij, op->coef, op->D, op->D2, op->gamma_dt};
}

int launch_leaf_assemble(const hps_op *op, double *W, hipStream_t st) {
    const int64_t tot = (int64_t)op->q2 * op->q2;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 64);
    hipLaunchKernelGGL(k_leaf_assemble, dim3(bx, build_leaves(op)), dim3(NT), 0, st, build_leaf_args(op), W);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_leaf_S(const hps_op *op, const double *ainv, double *S, hipStream_t st) {
    const int64_t tot = (int64_t)op->q2 * 4 * op->q;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 64);
    hipLaunchKernelGGL(k_leaf_S, dim3(bx, build_leaves(op)), dim3(NT), 0, st, build_leaf_args(op), ainv, S);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_leaf_T(const hps_op *op, const double *S, double *T, hipStream_t st) {
    const int64_t tot = (int64_t)16 * op->q * op->q;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 64);
    hipLaunchKernelGGL(k_leaf_T, dim3(bx, build_leaves(op)), dim3(NT), 0, st, build_leaf_args(op), S, T);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_leaf_assemble_cx(const hps_op *op, double *W, hipStream_t st) {
    const int64_t n = 2 * (int64_t)op->q2, tot = n * n;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 128);
    hipLaunchKernelGGL(k_leaf_assemble_cx, dim3(bx, build_leaves(op)), dim3(NT), 0, st, build_leaf_args(op), W);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_leaf_S_cx(const hps_op *op, const double *ainv, double *S, hipStream_t st) {
    const int64_t tot = 2 * (int64_t)op->q2 * 8 * op->q;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 128);
    hipLaunchKernelGGL(k_leaf_S_cx, dim3(bx, build_leaves(op)), dim3(NT), 0, st, build_leaf_args(op), ainv, S);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_leaf_T_cx(const hps_op *op, const double *S, double *T, hipStream_t st) {
    const int64_t tot = (int64_t)64 * op->q * op->q;
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 128);
    hipLaunchKernelGGL(k_leaf_T_cx, dim3(bx, build_leaves(op)), dim3(NT), 0, st, build_leaf_args(op), S, T);
    HPS_LAUNCHED();
    return HPS_OK;
}

int launch_merge_gather(const Level &L, int nodes, int64_t child_stride, bool root, const double *Tc, double *M,
                        double *B, double *Cm, double *Tn, hipStream_t st) {
    MergeArgs a{L.n1, L.n2, L.n3, L.n12, L.nbc, L.a1, L.a3, L.b2, L.b3, Tc, M, B, Cm, root ? nullptr : Tn, child_stride};
    const int64_t tot = (int64_t)L.n3 * L.n3 + 2 * (int64_t)L.n3 * L.n12 +
                        (root ? 0 : (int64_t)L.n12 * L.n12);
    const unsigned bx = (unsigned)std::min<int64_t>(nblk(tot), 4096);
    hipLaunchKernelGGL(k_merge_gather, dim3(bx, nodes), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

int gj_invert(double *W, double *out, int n, int nb, unsigned char *used, int *order,
              double *colbuf, double *rowbuf, int *sing, hipStream_t st) {
    const size_t lds = gj_reg_lds(n);
    const char *env = getenv("HPS_GJ_REG");   // "0": always the batched kernels
    const bool reg = !(env && env[0] == '0') && nb > 0 && n >= 1;
#define HPS_GJ_REG_CASE(RA, CB)                                                           \
    if (reg && n <= GJ_TR * (RA) && n <= GJ_TC * (CB)) {                                  \
        hipLaunchKernelGGL((k_gj_reg<RA, CB>), dim3(nb), dim3(GJ_NT), lds, st, (const double *)W, out, n, sing); \
        HPS_LAUNCHED();                                                                   \
        return HPS_OK;                                                                    \
    }
    HPS_GJ_REG_CASE(2, 1)
    HPS_GJ_REG_CASE(4, 2)
    HPS_GJ_REG_CASE(8, 4)
    HPS_GJ_REG_CASE(13, 7)
#undef HPS_GJ_REG_CASE
    HPS_HIP(hipMemsetAsync(used, 0, (size_t)n * nb, st));
    const int64_t tot = (int64_t)n * n * nb;
    const char *fenv = getenv("HPS_GJ_FUSED");   // "0": one pivot and one update launch per step
    if (fenv && fenv[0] == '0') {
        for (int k = 0; k < n; ++k) {
            hipLaunchKernelGGL(k_gj_pivot, dim3(nb), dim3(NT), 0, st, W, n, k, used, order, colbuf, rowbuf, sing);
            HPS_LAUNCHED();
            hipLaunchKernelGGL(k_gj_update, dim3(nblk(tot)), dim3(NT), 0, st, W, n, nb, k,
                               (const int *)order, (const double *)colbuf, (const double *)rowbuf);
            HPS_LAUNCHED();
        }
    } else {
        // the batch alternates between W and out (out holds no data before the end); the
        // column and row buffers hold two halves of n * nb, one per step parity
        const int64_t half = (int64_t)n * nb;
        hipLaunchKernelGGL(k_gj_pivot, dim3(nb), dim3(NT), 0, st, W, n, 0, used, order, colbuf, rowbuf, sing);
        HPS_LAUNCHED();
        double *buf[2] = {W, out};
        for (int k = 0; k < n; ++k) {
            const int npiv = k + 1 < n ? nb : 0;
            const int h = k & 1;
            hipLaunchKernelGGL(k_gj_step, dim3((unsigned)(npiv + nblk(tot))), dim3(NT), 0, st,
                               (const double *)buf[h], buf[h ^ 1], n, nb, k, npiv, used, order,
                               (const double *)(colbuf + h * half), (const double *)(rowbuf + h * half),
                               colbuf + (h ^ 1) * half, rowbuf + (h ^ 1) * half, sing);
            HPS_LAUNCHED();
        }
        // after n steps the batch is in buf[n & 1]; the unpermutation reads W
        if (n & 1) HPS_HIP(hipMemcpyAsync(W, out, sizeof(double) * tot, hipMemcpyDeviceToDevice, st));
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
                const double *src1, int ld1, int64_t stride1, hipStream_t st, double scale) {
    PackArgs a{};
    a.R = pn.R; a.C = pn.C; a.vw = pn.vw; a.rp = pn.rp; a.G = pn.G; a.S = pn.S;
    a.ntile = pn.ntile; a.kch = pn.kch;
    a.tile_elems = pn.tile_elems; a.node_elems = pn.node_elems;
    a.total = pn.node_elems * pn.nodes;
    a.src0 = src0; a.ld0 = ld0; a.stride0 = stride0; a.rows0 = rows0;
    a.src1 = src1; a.ld1 = ld1; a.stride1 = stride1;
    a.dst = pn.data;
    a.scale = scale;
    if (pn.vw == 2) hipLaunchKernelGGL(k_pack<double>, dim3(nblk(a.total)), dim3(NT), 0, st, a);
    else hipLaunchKernelGGL(k_pack<float>, dim3(nblk(a.total)), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

// every coefficient compared bitwise with its value at node 0
__global__ void k_coef_uniform(const double *coef, int64_t n, int *flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 5 * n) return;
    const int64_t c = t / n;
    if (__double_as_longlong(coef[t]) != __double_as_longlong(coef[c * n])) atomicOr(flag, 1);
}

int launch_coef_uniform(const double *coef, int64_t n, int *flag, hipStream_t st) {
    if (n <= 0) return HPS_OK;
    hipLaunchKernelGGL(k_coef_uniform, dim3(nblk(5 * n)), dim3(NT), 0, st, coef, n, flag);
    HPS_LAUNCHED();
    return HPS_OK;
}

}  // namespace hps
