// Composite operators of level pairs: the products of two adjacent tree levels of the
// merge formulas after eqs. (7)-(8) and of Algorithm 1 (Sec. 2.1), multiplied out once at
// build time so that one launch per direction sweeps both levels.
//
// Notation for an upper node tau (level l) with children alpha = 2 tau, beta = 2 tau + 1
// (level l + 1): X, U, S are the stored per-level operators (w3 = X d, h = [h1; h2] + U d,
// u3 = S u12 + w3); a1, a3, b2, b3 are the upper level's maps (tau's boundary m < n1 is
// alpha's boundary position a1[m], otherwise beta's b2[m - n1]; tau's J3 index k is alpha's
// position a3[k] and beta's b3[k]).
//
// Upward, with d_a, d_b the children's interface differences and e the node's difference
// of the fluxes its children pass through unchanged,
//   d_tau = e + U_b[b3, :] d_b - U_a[a3, :] d_a = V [d_a; d_b; e],  V = [-U_a[a3,:] | U_b[b3,:] | I],
// so [w3_a; w3_b; w3_tau; h_tau - pass-through] = M_up [d_a; d_b; e] with
//   M_up = [ X_a 0 0 ; 0 X_b 0 ; X_tau V ; [U_a[a1,:] | U_b[b2,:] | 0] (row blocks J1, J2) + U_tau V ].
// Downward, with the node's boundary values u12 and w3_tau,
//   u3_tau = S_tau u12 + w3_tau,
//   u3_a = S_a[:, a1] u12|J1 + S_a[:, a3] u3_tau + w3_a = ([S_a[:, a1 | 0]] + S_a[:, a3] [S_tau | I]) [u12; w3_tau] + w3_a,
// so M_dn = [ S_tau 0 ; S_a[:, a1 | 0] + S_a[:, a3] W ; S_b[:, 0 | b2] + S_b[:, b3] W ],  W = [S_tau | I],
// with the own-level w3 added when the rows are finalised.  The top pair takes the
// Dirichlet data f (the root's boundary values) and the differences below it:
//   u3_root = [S_root | X_root V] [f; d_a; d_b; e],  u3_a = [S_a[:, a1 | 0] | X_a | 0 | 0] [...] + S_a[:, a3] u3_root, ...
// The index tables that go with each composite are built here too (see PairArgs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "hps_internal.h"

using namespace hps;

namespace hps {

// dst[b][(c0 + j) * ldd + r0 + i] (+)= scale * src[b * sstr + cc * lds + rr], rr = ri ? ri[i] : i,
// cc = cj ? cj[j] : j; a negative index reads zero; src == null reads the identity.
struct PlaceArgs {
    double *dst;
    int ldd;
    int64_t dstr;
    int r0, c0, rows, cols;
    const double *src;
    int lds;
    int64_t sstr;
    const int *ri, *cj;
    double scale;
    int accumulate;
};

__global__ void k_place(PlaceArgs a) {
    const int64_t n = (int64_t)a.rows * a.cols;
    const int b = blockIdx.y;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % a.rows), j = (int)(t / a.rows);
        const int rr = a.ri ? a.ri[i] : i, cc = a.cj ? a.cj[j] : j;
        double v = 0.0;
        if (rr >= 0 && cc >= 0) v = a.src ? a.src[(int64_t)b * a.sstr + (int64_t)cc * a.lds + rr] : (rr == cc ? 1.0 : 0.0);
        double *d = a.dst + (int64_t)b * a.dstr + (int64_t)(a.c0 + j) * a.ldd + a.r0 + i;
        *d = a.accumulate ? *d + a.scale * v : a.scale * v;
    }
}

int launch_place(double *dst, int ldd, int64_t dstr, int r0, int c0, int rows, int cols, const double *src, int lds,
                 int64_t sstr, const int *ri, const int *cj, double scale, bool accumulate, int batch, hipStream_t st) {
    if (rows <= 0 || cols <= 0 || batch <= 0) return HPS_OK;
    PlaceArgs a{dst, ldd, dstr, r0, c0, rows, cols, src, lds, sstr, ri, cj, scale, accumulate ? 1 : 0};
    const int64_t n = (int64_t)rows * cols;
    const unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024);
    hipLaunchKernelGGL(k_place, dim3(gx, batch), dim3(NT), 0, st, a);
    HPS_LAUNCHED();
    return HPS_OK;
}

}  // namespace hps

namespace {

// grandchild offsets (relative to the node's four grandchildren, nbcc entries each) of
// alpha's / beta's boundary position j
struct Pos {
    const HostLevel &c;
    int nbcc;
    int a(int j) const { return j < c.n1 ? c.a1[j] : nbcc + c.b2[j - c.n1]; }
    int b(int j) const { return j < c.n1 ? 2 * nbcc + c.a1[j] : 3 * nbcc + c.b2[j - c.n1]; }
};

// host table to device memory: through the build's pinned staging when there is one (the
// copy stays in flight), else a plain copy that the caller waits for before the table dies
template <typename T>
int table_copy(const hps_op *op, T *dst, const std::vector<T> &v, hipStream_t st) {
    if (v.empty()) return HPS_OK;
    if (op->stage) return op->stage->copy(dst, v.data(), sizeof(T) * v.size());
    HPS_HIP(hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
    return HPS_OK;
}

// scratch allocated and freed in the stream's order (no device-wide wait)
struct DevScratch {
    hipStream_t st;
    std::vector<void *> p;
    explicit DevScratch(hipStream_t s) : st(s) {}
    ~DevScratch() {
        for (void *q : p) (void)hipFreeAsync(q, st);
    }
    template <typename T>
    int get(T **out, int64_t n) {
        void *q = nullptr;
        if (hipMallocAsync(&q, sizeof(T) * std::max<int64_t>(n, 1), st) != hipSuccess) {
            (void)hipGetLastError();
            hps_set_error("hipMallocAsync of %lld bytes for composite operators failed", (long long)(sizeof(T) * n));
            return HPS_ENOMEM;
        }
        p.push_back(q);
        *out = (T *)q;
        return HPS_OK;
    }
    template <typename T>
    int upload(const hps_op *op, T **out, const std::vector<T> &v) {
        TRY(get(out, (int64_t)v.size()));
        return table_copy(op, *out, v, st);
    }
};



int64_t level_nodes(int l) { return int64_t(1) << l; }

}  // namespace

// Workgroups a composite's launch is cut into: about two per compute unit.  A composite
// holds two levels' products, so thin tiles (the level panels' rule, at most 16 loads per
// lane) would take two rounds of workgroups; with two per compute unit every workgroup is
// resident at once and streams its longer rows (measured at 64x64 leaves, p = 16: 181 µs
// for both sweeps of a stage against 210 µs with the thin-tile rule and 210 µs per level).
static int pair_target() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    return 2 * cus;
}

// The packing of a composite: rows cut into tiles so that the launch has about `target`
// workgroups (at most NT / vw row vectors per tile: one row per thread); vw = 2 (FP64) or
// 4 (FP32)
static Panel pair_panel(int R, int C, int nodes, int target, int vw = 2) {
    // FP32 copies hold half the bytes per row: twice the workgroups (four per compute unit)
    // keep as many loads in flight (measured at 64x64 leaves, p = 16: FP32 sweeps of a
    // refined step 2.07 -> 1.92 ms; two, three, six, eight per unit were slower)
    if (vw == 4) target *= 2;
    const int RV = (R + vw - 1) / vw;
    const int per = std::max(1, (target + nodes - 1) / nodes);   // row tiles per node
    const int rp_max = std::min(NT / vw, std::max(1, (RV + per - 1) / per));
    return plan_panel(R, C, vw, nodes, rp_max, 0);
}

// Composites need one workgroup's input vector in LDS (no split-K), narrow level tiles
// and at least the root and one level below it.  Complex operators qualify too: their
// levels are the real embedding with two-component maps (the maps in hl are already
// doubled), which the composites multiply out like any real level pair.
bool hps::compose_eligible(const hps_op *op, const std::vector<HostLevel> &hl) {
    if ((op->flags & HPS_WIDE_TILES) || op->L < 2) return false;
    // the top pair (0, 1), then (2, 3), (4, 5), ... while the lower level exists
    for (int l = 0; l + 1 < op->L; l += 2) {
        const HostLevel &t = hl[l], &c = hl[l + 1];
        const int n12t = t.n1 + t.n2, nt = (int)level_nodes(l);
        const int CV = 2 * c.n3 + t.n3;
        if (l == 0) {
            if (pair_panel(t.n3 + 2 * c.n3, n12t + CV, 1, pair_target()).kch != 1) return false;
        } else if (pair_panel(CV + n12t, CV, nt, pair_target()).kch != 1 ||
                   pair_panel(t.n3 + 2 * c.n3, n12t + t.n3, nt, pair_target()).kch != 1) {
            return false;
        }
    }
    return true;
}

int hps::compose_pair(hps_op *op, int l, const std::vector<HostLevel> &hl, const double *Xc, const double *Uc,
                      const double *Sc, const double *Xt, const double *Ut, const double *St, hipStream_t st) {
    const HostLevel &T = hl[l], &Cl = hl[l + 1];
    const int n3t = T.n3, n1t = T.n1, n12t = T.n1 + T.n2;
    const int n3c = Cl.n3, n12c = Cl.n1 + Cl.n2;   // a child's boundary length = the child level's n12
    // grandchildren: level l + 2 nodes (or leaves), boundary length = the lower level's nbc
    const int nbcc = Cl.nbc;
    const Pos pos{Cl, nbcc};
    const int nt = (int)level_nodes(l);
    // uniform coefficients: one node's operators (children equal), composites stored once
    const bool uni = op->build_one;
    const int nb = uni ? 1 : nt;   // nodes whose composites are computed
    const bool top = (l == 0);
    DevScratch tmp(st);
    // index vectors on the device: the upper level's maps, padded to its boundary length
    std::vector<int> a1pad(n12t, -1), b2pad(n12t, -1);
    for (int m = 0; m < n1t; ++m) a1pad[m] = T.a1[m];
    for (int m = n1t; m < n12t; ++m) b2pad[m] = T.b2[m - n1t];
    int *d_a3, *d_b3, *d_a1pad, *d_b2pad;
    TRY(tmp.upload(op, &d_a3, T.a3));
    TRY(tmp.upload(op, &d_b3, T.b3));
    TRY(tmp.upload(op, &d_a1pad, a1pad));
    TRY(tmp.upload(op, &d_b2pad, b2pad));
    const int64_t sX = (int64_t)n3c * n3c, sU = (int64_t)n12c * n3c, sS = (int64_t)n3c * n12c;   // per child
    const int64_t cb = uni ? 0 : 1;   // the second child's operators follow the first's
    const double *Xa = Xc, *Xb = Xc + cb * sX, *Ua = Uc, *Ub = Uc + cb * sU, *Sa = Sc, *Sb = Sc + cb * sS;

    PairOps P;
    P.l = l;
    // V = [-U_a[a3,:] | U_b[b3,:] | I]  (n3t x (2 n3c + n3t)) per node
    const int CV = 2 * n3c + n3t;
    double *V;
    TRY(tmp.get(&V, (int64_t)n3t * CV * nb));
    const int64_t sV = (int64_t)n3t * CV;
    TRY(launch_place(V, n3t, sV, 0, 0, n3t, n3c, Ua, n12c, 2 * sU, d_a3, nullptr, -1.0, false, nb, st));
    TRY(launch_place(V, n3t, sV, 0, n3c, n3t, n3c, Ub, n12c, 2 * sU, d_b3, nullptr, 1.0, false, nb, st));
    TRY(launch_place(V, n3t, sV, 0, 2 * n3c, n3t, n3t, nullptr, 0, 0, nullptr, nullptr, 1.0, false, nb, st));
    // the children's S restricted to the upper node's J3 columns
    double *Sa3, *Sb3;
    TRY(tmp.get(&Sa3, (int64_t)n3c * n3t * nb));
    TRY(tmp.get(&Sb3, (int64_t)n3c * n3t * nb));
    const int64_t s3 = (int64_t)n3c * n3t;
    TRY(launch_place(Sa3, n3c, s3, 0, 0, n3c, n3t, Sa, n3c, 2 * sS, nullptr, d_a3, 1.0, false, nb, st));
    TRY(launch_place(Sb3, n3c, s3, 0, 0, n3c, n3t, Sb, n3c, 2 * sS, nullptr, d_b3, 1.0, false, nb, st));

    double *Mup = nullptr, *Mdn = nullptr;
    if (!top) {
        // ---- upward composite [w3_a; w3_b; w3_tau; h_tau] x [d_a; d_b; e] ----
        const int R = 2 * n3c + n3t + n12t, C = CV;
        const int64_t sM = (int64_t)R * C;
        TRY(tmp.get(&Mup, sM * nb));
        TRY(launch_zero(Mup, sM * nb, st));
        TRY(launch_place(Mup, R, sM, 0, 0, n3c, n3c, Xa, n3c, 2 * sX, nullptr, nullptr, 1.0, false, nb, st));
        TRY(launch_place(Mup, R, sM, n3c, n3c, n3c, n3c, Xb, n3c, 2 * sX, nullptr, nullptr, 1.0, false, nb, st));
        TRY(launch_dgemm(n3t, C, n3t, Xt, n3t, (int64_t)n3t * n3t, V, n3t, sV, Mup + 2 * n3c, R, sM, nb, 1.0, 0.0, st));
        const int h0 = 2 * n3c + n3t;
        TRY(launch_place(Mup, R, sM, h0, 0, n12t, n3c, Ua, n12c, 2 * sU, d_a1pad, nullptr, 1.0, false, nb, st));
        TRY(launch_place(Mup, R, sM, h0, n3c, n12t, n3c, Ub, n12c, 2 * sU, d_b2pad, nullptr, 1.0, false, nb, st));
        TRY(launch_dgemm(n12t, C, n3t, Ut, n12t, (int64_t)n12t * n3t, V, n3t, sV, Mup + h0, R, sM, nb, 1.0, 1.0, st));
        P.R_up = R;
        P.C_up = C;
        // ---- downward composite [u3_tau; u3_a; u3_b] x [u12; w3_tau] ----
        const int Rd = n3t + 2 * n3c, Cd = n12t + n3t;
        const int64_t sD = (int64_t)Rd * Cd;
        double *W;
        TRY(tmp.get(&W, (int64_t)n3t * Cd * nb));
        const int64_t sW = (int64_t)n3t * Cd;
        TRY(launch_place(W, n3t, sW, 0, 0, n3t, n12t, St, n3t, (int64_t)n3t * n12t, nullptr, nullptr, 1.0, false, nb, st));
        TRY(launch_place(W, n3t, sW, 0, n12t, n3t, n3t, nullptr, 0, 0, nullptr, nullptr, 1.0, false, nb, st));
        TRY(tmp.get(&Mdn, sD * nb));
        TRY(launch_zero(Mdn, sD * nb, st));
        TRY(launch_place(Mdn, Rd, sD, 0, 0, n3t, n12t, St, n3t, (int64_t)n3t * n12t, nullptr, nullptr, 1.0, false, nb,
                         st));
        TRY(launch_place(Mdn, Rd, sD, n3t, 0, n3c, n12t, Sa, n3c, 2 * sS, nullptr, d_a1pad, 1.0, false, nb, st));
        TRY(launch_place(Mdn, Rd, sD, n3t + n3c, 0, n3c, n12t, Sb, n3c, 2 * sS, nullptr, d_b2pad, 1.0, false, nb, st));
        TRY(launch_dgemm(n3c, Cd, n3t, Sa3, n3c, s3, W, n3t, sW, Mdn + n3t, Rd, sD, nb, 1.0, 1.0, st));
        TRY(launch_dgemm(n3c, Cd, n3t, Sb3, n3c, s3, W, n3t, sW, Mdn + n3t + n3c, Rd, sD, nb, 1.0, 1.0, st));
        P.R_dn = Rd;
        P.C_dn = Cd;
    } else {
        // ---- the top pair: [u3_root; u3_a; u3_b] x [f; d_a; d_b; e] ----
        const int R = n3t + 2 * n3c, C = n12t + CV;
        const int64_t sM = (int64_t)R * C;
        TRY(tmp.get(&Mdn, sM));
        TRY(launch_zero(Mdn, sM, st));
        TRY(launch_place(Mdn, R, sM, 0, 0, n3t, n12t, St, n3t, 0, nullptr, nullptr, 1.0, false, 1, st));
        TRY(launch_dgemm(n3t, CV, n3t, Xt, n3t, 0, V, n3t, 0, Mdn + (int64_t)n12t * R, R, 0, 1, 1.0, 0.0, st));
        TRY(launch_place(Mdn, R, sM, n3t, 0, n3c, n12t, Sa, n3c, 0, nullptr, d_a1pad, 1.0, false, 1, st));
        TRY(launch_place(Mdn, R, sM, n3t, n12t, n3c, n3c, Xa, n3c, 0, nullptr, nullptr, 1.0, false, 1, st));
        TRY(launch_place(Mdn, R, sM, n3t + n3c, 0, n3c, n12t, Sb, n3c, 0, nullptr, d_b2pad, 1.0, false, 1, st));
        TRY(launch_place(Mdn, R, sM, n3t + n3c, n12t + n3c, n3c, n3c, Xb, n3c, 0, nullptr, nullptr, 1.0, false, 1, st));
        // the children's rows: + S_a[:, a3] u3_root (the root rows, already complete)
        TRY(launch_dgemm(n3c, C, n3t, Sa3, n3c, 0, Mdn, R, 0, Mdn + n3t, R, 0, 1, 1.0, 1.0, st));
        TRY(launch_dgemm(n3c, C, n3t, Sb3, n3c, 0, Mdn, R, 0, Mdn + n3t + n3c, R, 0, 1, 1.0, 1.0, st));
        P.R_dn = R;
        P.C_dn = C;
    }

    // ---- pack (streaming layout, FP64) ----
    const int target = pair_target();
    auto pack = [&](Panel &pn, const double *M, int R, int C, int vw) -> int {
        pn = pair_panel(R, C, nt, target, vw);
        if (uni) pn = shared_panel(pn);
        void *d;
        if (hipMalloc(&d, (vw == 2 ? 8 : 4) * pn.node_elems * pn.nodes) != hipSuccess) {
            (void)hipGetLastError();
            hps_set_error("hipMalloc for a composite operator failed");
            return HPS_ENOMEM;
        }
        op->allocs.push_back(d);
        op->operator_bytes += pn.bytes();
        op->total_bytes += pn.bytes();
        pn.data = d;
        if (pn.kch != 1 || pn.rp * pn.vw > NT) {
            hps_set_error("internal: a composite operator was planned with column chunks");
            return HPS_EDEVICE;
        }
        return launch_pack(pn, M, R, (int64_t)R * C, R, nullptr, 0, 0, st);
    };
    if (!top) TRY(pack(P.up, Mup, P.R_up, P.C_up, 2));
    TRY(pack(P.dn, Mdn, P.R_dn, P.C_dn, 2));
    if (op->flags & HPS_FP32_IR) {   // the FP32 sweeps' copies, rounded from the same products
        if (!top) TRY(pack(P.up32, Mup, P.R_up, P.C_up, 4));
        TRY(pack(P.dn32, Mdn, P.R_dn, P.C_dn, 4));
    }

    // ---- index tables ----
    std::vector<int> tab;
    auto put = [&](const std::vector<int> &v) {
        const int off = (int)tab.size();
        tab.insert(tab.end(), v.begin(), v.end());
        return off;
    };
    const int Cg = top ? P.C_dn : P.C_up;    // columns of the gather from the grandchildren's fluxes
    const int g0 = top ? n12t : 0;           // the first such column
    std::vector<int> plus(Cg, 0), minus(Cg, 0), j3(Cg, 0);
    for (int k = 0; k < n3c; ++k) {
        plus[g0 + k] = nbcc + Cl.b3[k];
        minus[g0 + k] = Cl.a3[k];
        j3[g0 + k] = k;
        plus[g0 + n3c + k] = 3 * nbcc + Cl.b3[k];
        minus[g0 + n3c + k] = 2 * nbcc + Cl.a3[k];
        j3[g0 + n3c + k] = n3c + k;
    }
    for (int k = 0; k < n3t; ++k) {
        plus[g0 + 2 * n3c + k] = pos.b(T.b3[k]);
        minus[g0 + 2 * n3c + k] = pos.a(T.a3[k]);
        j3[g0 + 2 * n3c + k] = -(k + 1);
    }
    P.t_plus = put(plus);
    P.t_minus = put(minus);
    P.t_j3 = put(j3);
    if (!top) {
        std::vector<int> fin(3 * (size_t)P.R_up, 0);
        for (int r = 0; r < P.R_up; ++r) {
            int kind, idx, pass = 0;
            if (r < 2 * n3c) {
                kind = 0;
                idx = r;
            } else if (r < 2 * n3c + n3t) {
                kind = 1;
                idx = r - 2 * n3c;
            } else {
                kind = 2;
                idx = r - 2 * n3c - n3t;
                pass = idx < n1t ? pos.a(T.a1[idx]) : pos.b(T.b2[idx - n1t]);
            }
            fin[3 * r] = kind;
            fin[3 * r + 1] = idx;
            fin[3 * r + 2] = pass;
        }
        P.t_fin_up = put(fin);
    }
    {
        std::vector<int> fin(4 * (size_t)P.R_dn, 0);
        for (int r = 0; r < P.R_dn; ++r) {
            int kind, idx, p1, p2;
            if (r < n3t) {
                kind = top ? -1 : 1;
                idx = r;
                p1 = pos.a(T.a3[r]);
                p2 = pos.b(T.b3[r]);
            } else if (r < n3t + n3c) {
                const int k = r - n3t;
                kind = top ? -1 : 0;
                idx = k;
                p1 = Cl.a3[k];
                p2 = nbcc + Cl.b3[k];
            } else {
                const int k = r - n3t - n3c;
                kind = top ? -1 : 0;
                idx = n3c + k;
                p1 = 2 * nbcc + Cl.a3[k];
                p2 = 3 * nbcc + Cl.b3[k];
            }
            fin[4 * r] = kind;
            fin[4 * r + 1] = idx;
            fin[4 * r + 2] = p1;
            fin[4 * r + 3] = p2;
        }
        P.t_fin_dn = put(fin);
    }
    {
        std::vector<int> copy(n12t);
        for (int m = 0; m < n12t; ++m) copy[m] = m < n1t ? pos.a(T.a1[m]) : pos.b(T.b2[m - n1t]);
        P.t_copy = put(copy);
    }
    int *d_tab;
    if (hipMalloc(&d_tab, sizeof(int) * tab.size()) != hipSuccess) {
        (void)hipGetLastError();
        hps_set_error("hipMalloc for composite tables failed");
        return HPS_ENOMEM;
    }
    op->allocs.push_back(d_tab);
    TRY(table_copy(op, d_tab, tab, st));
    P.tab = d_tab;
    // without the build's staging the host tables above die at return while their copies
    // may still be in flight (the device scratch is freed in stream order either way)
    if (!op->stage) HPS_HIP(hipStreamSynchronize(st));
    op->pairs.push_back(P);
    return HPS_OK;
}

// ---------------------------------------------------------------------------------------
// The direct sweep of a small tree.  With no boundary or jump data the interface values
// the level sweeps produce are a linear function of the leaves' particular fluxes h alone
// (Algorithm 1 of Sec. 2.1: every merge and every downward step is linear in h), so for a
// small tree the whole sweep -- 2 L - 1 or its composite-pair launches -- is one product
// M h.  M is taken column by column from the operator's own sweeps of unit vectors, so it
// is the map the sweeps compute, up to rounding.
// ---------------------------------------------------------------------------------------
namespace {

__global__ void k_unit(double *v, int64_t n, int64_t k) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        v[t] = t == k ? 1.0 : 0.0;
}

// column c of M: the interface values, read at each row's first leaf-boundary slot
__global__ void k_take_col(const double *ub, const int *rows, int R, double *col) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) col[r] = ub[rows[2 * r]];
}

constexpr int64_t kDirectMaxBytes = int64_t(2) << 20;   // M of at most 2 MiB

}  // namespace

int hps::build_direct(hps_op *op, hipStream_t st) {
    const char *env = std::getenv("HPS_DIRECT");
    if (env && env[0] == '0') return HPS_OK;
    if (op->ncomp != 1 || (op->flags & (HPS_FP32_IR | HPS_WIDE_TILES)) || op->L < 2 || op->n_iface <= 0) return HPS_OK;
    const int q = op->q, n1 = op->grid.n1, n2 = op->grid.n2, nb = 4 * q;
    const int64_t R = op->n_iface, C = (int64_t)op->nleaves * nb;
    if (R * C * 8 > kDirectMaxBytes) return HPS_OK;
    // leaf-boundary slots: heap leaf of each leaf (i, j), the two slots of each interface
    // node (canonical interface order: vertical lines first), the domain-boundary slots
    std::vector<int> ij(2 * (size_t)op->nleaves), heap((size_t)n1 * n2);
    HPS_HIP(hipMemcpy(ij.data(), op->leaf_ij, sizeof(int) * ij.size(), hipMemcpyDeviceToHost));
    for (int h = 0; h < op->nleaves; ++h) heap[(size_t)ij[2 * h + 1] * n1 + ij[2 * h]] = h;
    auto slot = [&](int i, int j, int e, int m) { return heap[(size_t)j * n1 + i] * nb + e * q + m; };
    std::vector<int> rows(2 * (size_t)R), zero;
    const int64_t nv = (int64_t)(n1 - 1) * n2 * q;
    for (int64_t t = 0; t < R; ++t) {
        if (t < nv) {
            const int k = (int)(t / ((int64_t)n2 * q)) + 1, rem = (int)(t % ((int64_t)n2 * q));
            rows[2 * t] = slot(k - 1, rem / q, 1, rem % q);
            rows[2 * t + 1] = slot(k, rem / q, 0, rem % q);
        } else {
            const int64_t u = t - nv;
            const int k = (int)(u / ((int64_t)n1 * q)) + 1, rem = (int)(u % ((int64_t)n1 * q));
            rows[2 * t] = slot(rem / q, k - 1, 3, rem % q);
            rows[2 * t + 1] = slot(rem / q, k, 2, rem % q);
        }
    }
    for (int j = 0; j < n2; ++j)
        for (int i = 0; i < n1; ++i)
            for (int m = 0; m < q; ++m) {
                if (i == 0) zero.push_back(slot(i, j, 0, m));
                if (i == n1 - 1) zero.push_back(slot(i, j, 1, m));
                if (j == 0) zero.push_back(slot(i, j, 2, m));
                if (j == n2 - 1) zero.push_back(slot(i, j, 3, m));
            }
    // the streaming layout: about two row tiles' workgroups per compute unit; a row longer
    // than one workgroup's LDS holds keeps the level sweeps
    Panel pn = pair_panel((int)R, (int)C, 1, pair_target(), 2);
    if (pn.kch != 1 || pn.rp * pn.vw > NT) return HPS_OK;
    // the slot tables, kept with the operator
    auto keep = [&](const std::vector<int> &v, int **out) -> int {
        if (hipMalloc(out, sizeof(int) * std::max<size_t>(v.size(), 1)) != hipSuccess) {
            (void)hipGetLastError();
            hps_set_error("hipMalloc for the direct sweep tables failed");
            return HPS_ENOMEM;
        }
        op->allocs.push_back(*out);
        op->total_bytes += (int64_t)(sizeof(int) * v.size());
        if (!v.empty()) HPS_HIP(hipMemcpyAsync(*out, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice, st));
        return HPS_OK;
    };
    TRY(keep(rows, &op->d_rows));
    TRY(keep(zero, &op->d_zero));
    op->n_zero = (int)zero.size();
    void *d = nullptr;
    if (hipMalloc(&d, 8 * pn.node_elems) != hipSuccess) {
        (void)hipGetLastError();
        hps_set_error("hipMalloc for the direct sweep operator failed");
        return HPS_ENOMEM;
    }
    op->allocs.push_back(d);
    op->operator_bytes += pn.bytes();
    op->total_bytes += pn.bytes();
    pn.data = d;
    // M column by column: the operator's FP64 sweep of each unit flux vector
    DevScratch tmp(st);
    double *M = nullptr;
    TRY(tmp.get(&M, R * C));
    const unsigned gz = (unsigned)std::min<int64_t>((C + NT - 1) / NT, 1024), gr = (unsigned)((R + NT - 1) / NT);
    for (int64_t c = 0; c < C; ++c) {
        hipLaunchKernelGGL(k_unit, dim3(gz), dim3(NT), 0, st, op->h_leaf, C, c);
        HPS_LAUNCHED();
        TRY(launch_levels(op, false, nullptr, nullptr, st));
        hipLaunchKernelGGL(k_take_col, dim3(gr), dim3(NT), 0, st, (const double *)op->ub_leaf,
                           (const int *)op->d_rows, (int)R, M + c * R);
        HPS_LAUNCHED();
    }
    TRY(launch_pack(pn, M, (int)R, R * C, (int)R, nullptr, 0, 0, st));
    HPS_HIP(hipStreamSynchronize(st));   // the scratch M is freed on return
    op->dpn = pn;
    op->direct = true;
    return HPS_OK;
}
