// Host side of the C ABI: argument checking, the tree plan, the GPU build and the
// stage-solve / time-step drivers.  Every arithmetic step of the build and of the solves
// runs in the kernels of hps_kernels.hip; this file only plans, allocates and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hps_internal.h"

using namespace hps;

// ---------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------
static thread_local char g_err[1024] = "no error";

void hps_set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

extern "C" const char *hps_last_error(void) { return g_err; }


// ---------------------------------------------------------------------------------------
// grid
// ---------------------------------------------------------------------------------------
static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static int check_grid(const hps_grid *g) {
    CHECK_ARG(g != nullptr, "grid is NULL");
    CHECK_ARG(is_pow2(g->n1) && is_pow2(g->n2), "n1 and n2 must be powers of two (got %d, %d)", g->n1, g->n2);
    CHECK_ARG((int64_t)g->n1 * g->n2 <= (1 << 14), "at most 2^14 leaves are supported");
    CHECK_ARG(g->p >= 3 && g->p <= PMAX, "p must be in [3, %d] (got %d)", PMAX, g->p);
    CHECK_ARG(std::isfinite(g->x0) && std::isfinite(g->x1) && std::isfinite(g->y0) && std::isfinite(g->y1),
              "domain bounds must be finite");
    CHECK_ARG(g->x1 > g->x0 && g->y1 > g->y0, "empty domain");
    const double hx = (g->x1 - g->x0) / g->n1, hy = (g->y1 - g->y0) / g->n2;
    CHECK_ARG(std::fabs(hx - hy) <= 1e-12 * std::max(std::fabs(hx), std::fabs(hy)),
              "leaves must be square: (x1-x0)/n1 = %.17g, (y1-y0)/n2 = %.17g", hx, hy);
    return HPS_OK;
}

struct Counts {
    int64_t N, n_int, n_vert, n_horz, n_edge, n_bdry, n_iface;
};

static Counts counts(const hps_grid *g) {
    Counts c{};
    const int64_t q = g->p - 2, n1 = g->n1, n2 = g->n2;
    c.n_int = n1 * n2 * q * q;
    c.n_vert = (n1 + 1) * n2 * q;
    c.n_horz = (n2 + 1) * n1 * q;
    c.n_edge = c.n_vert + c.n_horz;
    c.N = c.n_int + c.n_edge;
    c.n_bdry = 2 * q * (n1 + n2);
    c.n_iface = c.n_edge - c.n_bdry;
    return c;
}

extern "C" int64_t hps_num_nodes(const hps_grid *grid, int64_t *n_int, int64_t *n_iface, int64_t *n_bdry) {
    int rc = check_grid(grid);
    if (rc) return rc;
    Counts c = counts(grid);
    if (n_int) *n_int = c.n_int;
    if (n_iface) *n_iface = c.n_iface;
    if (n_bdry) *n_bdry = c.n_bdry;
    return c.N;
}

// Chebyshev-Lobatto offsets on [0, h]: h (1 - cos(m pi / (p-1))) / 2, ascending in m.
static double cheb_offset(double h, int m, int p) {
    return h * (1.0 - std::cos(M_PI * m / (p - 1))) / 2.0;
}

extern "C" int hps_nodes(const hps_grid *g, double *x, double *y) {
    TRY(check_grid(g));
    CHECK_ARG(x && y, "x and y must be host arrays of N doubles");
    const Counts c = counts(g);
    const int q = g->p - 2, n1 = g->n1, n2 = g->n2, p = g->p;
    const double h = (g->x1 - g->x0) / n1;
    for (int j = 0; j < n2; ++j)
        for (int i = 0; i < n1; ++i)
            for (int b = 1; b <= q; ++b)
                for (int a = 1; a <= q; ++a) {
                    const int64_t k = ((int64_t)(j * n1 + i) * q + (b - 1)) * q + (a - 1);
                    x[k] = (g->x0 + i * h) + cheb_offset(h, a, p);
                    y[k] = (g->y0 + j * h) + cheb_offset(h, b, p);
                }
    for (int k = 0; k <= n1; ++k)
        for (int j = 0; j < n2; ++j)
            for (int m = 0; m < q; ++m) {
                const int64_t idx = c.n_int + ((int64_t)k * n2 + j) * q + m;
                x[idx] = g->x0 + k * h;
                y[idx] = (g->y0 + j * h) + cheb_offset(h, m + 1, p);
            }
    for (int k = 0; k <= n2; ++k)
        for (int i = 0; i < n1; ++i)
            for (int m = 0; m < q; ++m) {
                const int64_t idx = c.n_int + c.n_vert + ((int64_t)k * n1 + i) * q + m;
                x[idx] = (g->x0 + i * h) + cheb_offset(h, m + 1, p);
                y[idx] = g->y0 + k * h;
            }
    return HPS_OK;
}

// Derivative on the physical nodes of one leaf (side h), row-major D[a*p + m]:
// Chebyshev-Gauss-Lobatto collocation derivative on xi_m = cos(m pi/(p-1)) scaled by
// dxi/dx = -2/h; off-diagonal (k_i/k_j)(-1)^(i+j)/(xi_i - xi_j), k = 2 at the ends,
// diagonal = minus the off-diagonal row sum.
static void leaf_derivative(int p, double h, std::vector<double> &D, std::vector<double> &D2) {
    std::vector<double> xi(p);
    for (int m = 0; m < p; ++m) xi[m] = std::cos(M_PI * m / (p - 1));
    D.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) {
        double rs = 0.0;
        for (int j = 0; j < p; ++j) {
            if (i == j) continue;
            const double ki = (i == 0 || i == p - 1) ? 2.0 : 1.0;
            const double kj = (j == 0 || j == p - 1) ? 2.0 : 1.0;
            const double sgn = ((i + j) % 2) ? -1.0 : 1.0;
            const double v = (ki / kj) * sgn / (xi[i] - xi[j]);
            D[(size_t)i * p + j] = v;
            rs += v;
        }
        D[(size_t)i * p + i] = -rs;
    }
    for (auto &v : D) v *= -2.0 / h;
    D2.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            double s = 0.0;
            for (int m = 0; m < p; ++m) s += D[(size_t)i * p + m] * D[(size_t)m * p + j];
            D2[(size_t)i * p + j] = s;
        }
}

// ---------------------------------------------------------------------------------------
// panel planning
// ---------------------------------------------------------------------------------------
namespace hps {
Panel plan_panel(int R, int C, int vw, int nodes, int rp_max, int min_wg) {
    Panel p;
    p.R = R; p.C = C; p.vw = vw; p.nodes = nodes;
    const int RV = (R + vw - 1) / vw;
    p.ntile = (RV + rp_max - 1) / rp_max;
    // more, thinner row tiles until the sweep has min_wg workgroups: the column groups of
    // a workgroup are reduced in LDS, so no cross-workgroup reduction is needed
    if (min_wg > 0 && (int64_t)nodes * p.ntile < min_wg)
        p.ntile = (int)std::min<int64_t>(RV, (min_wg + nodes - 1) / nodes);
    p.rp = (RV + p.ntile - 1) / p.ntile;
    // level panels: at most 16 loads per lane, so a workgroup issues its whole block up front
    if (min_wg > 0)
        while (p.rp > 1 && (int64_t)(C + NT / p.rp - 1) / (NT / p.rp) > 16) p.rp = (p.rp + 1) / 2;
    p.ntile = (RV + p.rp - 1) / p.rp;
    const int Gmax = std::max(1, NT / p.rp);
    // column groups: fewest padded columns, then most groups (narrow panels may leave
    // lanes idle rather than stream padding)
    int bestG = Gmax;
    int64_t bestPad = -1;
    for (int G = Gmax; G >= std::max(1, std::min(Gmax / 2, C)); --G) {
        const int64_t pad = (int64_t)((C + G - 1) / G) * G - C;
        if (bestPad < 0 || pad < bestPad) {
            bestPad = pad;
            bestG = G;
        }
    }
    p.G = bestG;
    // column chunks only when one workgroup's input vector would not fit in LDS
    p.kch = 1;
    while ((int64_t)((C + p.G * p.kch - 1) / (p.G * p.kch)) * p.G * (vw == 2 ? 8 : 4) > XS_BYTES) ++p.kch;
    p.S = (C + p.G * p.kch - 1) / (p.G * p.kch);
    p.tile_elems = (int64_t)p.S * p.G * p.rp * vw;
    p.node_elems = (int64_t)p.ntile * p.kch * p.tile_elems;
    return p;
}

Panel shared_panel(Panel p) {
    p.nodes = 1;
    p.shared = true;
    return p;
}

// Workgroups a level's product is cut into at least: enough to fill the GPU for one
// problem, or (HPS_WIDE_TILES) few and large when many problems share each launch.
// mwg > 0: the number chosen by the autotuner for this operator class.
static int level_min_wg(int flags, int mwg = 0) {
    if (mwg > 0) return mwg;
    return (flags & HPS_WIDE_TILES) ? 32 : 1024;
}

// Bytes of the packed operators hps_build stores for a grid, from the same panel plans
// (the tree splits the longer side of each box, ties with a vertical cut).
int64_t plan_operator_bytes(const hps_grid &g, int flags, int ncomp, int mwg) {
    const int q = g.p - 2, q2 = q * q * ncomp, nl = g.n1 * g.n2;
    const bool ir = (flags & HPS_FP32_IR) != 0;
    const bool uni = (flags & HPS_UNIFORM_COEFFS) != 0;
    auto sh = [&](const Panel &p) { return uni ? shared_panel(p) : p; };
    const int nbl = 4 * q * ncomp;
    int64_t bytes = sh(plan_panel(q2, q2, 2, nl, 256, 0)).bytes() + sh(plan_panel(q2, nbl, 2, nl, 256, 0)).bytes();
    if (ir)
        bytes += sh(plan_panel(q2, q2, 4, nl, 256, 0)).bytes() + sh(plan_panel(q2, nbl, 4, nl, 256, 0)).bytes();
    int w = g.n1, h = g.n2, nodes = 1;
    bool root = true;
    while (w * h > 1) {
        const bool vert = w >= h;
        const int n3 = q * (vert ? h : w) * ncomp, n12 = 2 * q * (w + h) * ncomp;
        const int rows = root ? n3 : n3 + n12;
        const int lmw = level_min_wg(flags, mwg);
        bytes += sh(plan_panel(rows, n3, 2, nodes, 64, lmw)).bytes() + sh(plan_panel(n3, n12, 2, nodes, 64, lmw)).bytes();
        if (ir)
            bytes += sh(plan_panel(rows, n3, 4, nodes, 64, lmw)).bytes() +
                     sh(plan_panel(n3, n12, 4, nodes, 64, lmw)).bytes();
        if (vert) w /= 2;
        else h /= 2;
        nodes *= 2;
        root = false;
    }
    return bytes;
}
}  // namespace hps

// ---------------------------------------------------------------------------------------
// allocation helpers
// ---------------------------------------------------------------------------------------
template <typename T>
static int dev_alloc(hps_op *op, T **ptr, int64_t n, bool track = true) {
    *ptr = nullptr;
    if (n <= 0) n = 1;
    hipError_t e = hipMalloc((void **)ptr, sizeof(T) * (size_t)n);
    if (e != hipSuccess) {
        hps_set_error("hipMalloc of %lld bytes failed: %s", (long long)(sizeof(T) * n), hipGetErrorString(e));
        *ptr = nullptr;
        return HPS_ENOMEM;
    }
    if (track && op) {
        op->allocs.push_back(*ptr);
        op->total_bytes += (int64_t)sizeof(T) * n;
    }
    return HPS_OK;
}

hps::HostStage::~HostStage() {
    if (!chunks.empty()) (void)hipStreamSynchronize(st);
    for (void *c : chunks) (void)hipHostFree(c);
}

int hps::HostStage::copy(void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return HPS_OK;
    if (chunks.empty() || used + bytes > cap) {
        const size_t want = std::max<size_t>(bytes, size_t(8) << 20);
        void *c = nullptr;
        if (hipHostMalloc(&c, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            hps_set_error("hipHostMalloc of %zu bytes for the build's staging failed", want);
            return HPS_ENOMEM;
        }
        chunks.push_back(c);
        used = 0;
        cap = want;
    }
    unsigned char *p = static_cast<unsigned char *>(chunks.back()) + used;
    std::memcpy(p, src, bytes);
    used += (bytes + 255) & ~size_t(255);
    HPS_HIP(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, st));
    return HPS_OK;
}

template <typename T>
static int upload(hps_op *op, T **ptr, const std::vector<T> &v, hipStream_t st) {
    TRY(dev_alloc(op, ptr, (int64_t)v.size()));
    if (v.empty()) return HPS_OK;
    if (op->stage) return op->stage->copy(*ptr, v.data(), sizeof(T) * v.size());
    HPS_HIP(hipMemcpyAsync(*ptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
    return HPS_OK;
}

// device scratch of the build, allocated and freed in stream order (a plain hipFree would
// wait for the whole device), freed at scope exit at the latest
struct TempBuf {
    hipStream_t st;
    std::vector<void *> ptrs;
    explicit TempBuf(hipStream_t s) : st(s) {}
    ~TempBuf() {
        for (void *p : ptrs) (void)hipFreeAsync(p, st);
    }
    template <typename T>
    int get(T **ptr, int64_t n) {
        *ptr = nullptr;
        const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(n, 1);
        if (hipMallocAsync((void **)ptr, bytes, st) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            hps_set_error("hipMallocAsync of %zu bytes of build scratch failed", bytes);
            return HPS_ENOMEM;
        }
        ptrs.push_back(*ptr);
        return HPS_OK;
    }
    void release(void *p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            (void)hipFreeAsync(*it, st);
            ptrs.erase(it);
        }
    }
};

int check_device_ptr(const void *p, const char *name) {
    if (!p) return HPS_OK;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess || (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        hps_set_error("%s must be a device pointer", name);
        return HPS_EINVAL;
    }
    return HPS_OK;
}

static int alloc_panel(hps_op *op, Panel &pn) {
    if (pn.vw == 2) {
        double *d;
        TRY(dev_alloc(op, &d, pn.node_elems * pn.nodes));
        pn.data = d;
    } else {
        float *f;
        TRY(dev_alloc(op, &f, pn.node_elems * pn.nodes));
        pn.data = f;
    }
    op->operator_bytes += pn.bytes();
    return HPS_OK;
}

// ---------------------------------------------------------------------------------------
// tree plan (host): boxes, boundaries in node order, J1/J2/J3 maps per level
// ---------------------------------------------------------------------------------------
struct Box {
    int i0, i1, j0, j1;
};


static int plan_tree(const hps_op *op, std::vector<int> &leaf_ij, std::vector<HostLevel> &hl,
                     std::vector<int> &root_map, std::vector<int> &bnd_glob) {
    const hps_grid &g = op->grid;
    const int n1 = g.n1, n2 = g.n2, q = op->q, L = op->L;
    // boxes, heap order per level
    std::vector<std::vector<Box>> boxes(L + 1);
    boxes[0].push_back(Box{0, n1, 0, n2});
    for (int l = 0; l < L; ++l) {
        for (const Box &b : boxes[l]) {
            if (b.i1 - b.i0 >= b.j1 - b.j0) {   // halve the longer side, ties cut vertically
                const int im = (b.i0 + b.i1) / 2;
                boxes[l + 1].push_back(Box{b.i0, im, b.j0, b.j1});
                boxes[l + 1].push_back(Box{im, b.i1, b.j0, b.j1});
            } else {
                const int jm = (b.j0 + b.j1) / 2;
                boxes[l + 1].push_back(Box{b.i0, b.i1, b.j0, jm});
                boxes[l + 1].push_back(Box{b.i0, b.i1, jm, b.j1});
            }
        }
    }
    leaf_ij.resize(2 * (size_t)op->nleaves);
    for (int k = 0; k < op->nleaves; ++k) {
        const Box &b = boxes[L][k];
        if (b.i1 - b.i0 != 1 || b.j1 - b.j0 != 1) {
            hps_set_error("internal: tree leaves are not single squares");
            return HPS_EINVAL;
        }
        leaf_ij[2 * k] = b.i0;
        leaf_ij[2 * k + 1] = b.j0;
    }
    auto vert = [&](int k, int j, int m) { return op->n_int + ((int64_t)k * n2 + j) * q + m; };
    auto horz = [&](int k, int i, int m) { return op->n_int + op->n_vert + ((int64_t)k * n1 + i) * q + m; };
    // interface / boundary index of every edge node (or -1)
    std::vector<int> iface(op->n_edge, -1), bpos(op->n_edge, -1);
    bnd_glob.assign(op->n_bdry, 0);
    {
        int64_t ni = 0, nb = 0;
        for (int k = 0; k <= n1; ++k)
            for (int j = 0; j < n2; ++j)
                for (int m = 0; m < q; ++m) {
                    const int64_t e = vert(k, j, m) - op->n_int;
                    if (k == 0 || k == n1) {
                        bpos[e] = (int)nb;
                        bnd_glob[nb++] = (int)(e + op->n_int);
                    } else {
                        iface[e] = (int)ni++;
                    }
                }
        for (int k = 0; k <= n2; ++k)
            for (int i = 0; i < n1; ++i)
                for (int m = 0; m < q; ++m) {
                    const int64_t e = horz(k, i, m) - op->n_int;
                    if (k == 0 || k == n2) {
                        bpos[e] = (int)nb;
                        bnd_glob[nb++] = (int)(e + op->n_int);
                    } else {
                        iface[e] = (int)ni++;
                    }
                }
        if (ni != op->n_iface || nb != op->n_bdry) {
            hps_set_error("internal: edge classification mismatch");
            return HPS_EINVAL;
        }
    }
    // boundaries in node order, bottom-up; leaf order [left, right, bottom, top]
    std::vector<std::vector<int64_t>> cur(op->nleaves), nxt;
    for (int k = 0; k < op->nleaves; ++k) {
        const int i = leaf_ij[2 * k], j = leaf_ij[2 * k + 1];
        auto &v = cur[k];
        v.reserve(4 * q);
        for (int m = 0; m < q; ++m) v.push_back(vert(i, j, m));
        for (int m = 0; m < q; ++m) v.push_back(vert(i + 1, j, m));
        for (int m = 0; m < q; ++m) v.push_back(horz(j, i, m));
        for (int m = 0; m < q; ++m) v.push_back(horz(j + 1, i, m));
    }
    hl.assign(L, HostLevel{});
    std::vector<int> posB(op->n_edge, -1);
    std::vector<char> in3(op->n_edge, 0);
    for (int l = L - 1; l >= 0; --l) {
        const int nodes = 1 << l;
        nxt.assign(nodes, {});
        HostLevel &H = hl[l];
        for (int k = 0; k < nodes; ++k) {
            const auto &A = cur[2 * k], &B = cur[2 * k + 1];
            if (A.size() != B.size()) {
                hps_set_error("internal: children of one node differ in boundary length");
                return HPS_EINVAL;
            }
            for (size_t t = 0; t < B.size(); ++t) posB[B[t] - op->n_int] = (int)t;
            std::vector<int> a1, a3, b2, b3;
            std::vector<int64_t> J3;
            for (size_t t = 0; t < A.size(); ++t) {
                const int64_t e = A[t] - op->n_int;
                if (posB[e] >= 0) {
                    a3.push_back((int)t);
                    b3.push_back(posB[e]);
                    J3.push_back(A[t]);
                    in3[e] = 1;
                } else {
                    a1.push_back((int)t);
                }
            }
            for (size_t t = 0; t < B.size(); ++t)
                if (!in3[B[t] - op->n_int]) b2.push_back((int)t);
            auto &nb = nxt[k];
            nb.reserve(a1.size() + b2.size());
            for (int t : a1) nb.push_back(A[t]);
            for (int t : b2) nb.push_back(B[t]);
            if (k == 0) {
                H.a1 = a1; H.a3 = a3; H.b2 = b2; H.b3 = b3;
                H.n1 = (int)a1.size(); H.n2 = (int)b2.size(); H.n3 = (int)a3.size();
                H.nbc = (int)A.size();
                H.j3i.assign((size_t)nodes * H.n3, 0);
            } else if (a1 != H.a1 || a3 != H.a3 || b2 != H.b2 || b3 != H.b3) {
                hps_set_error("internal: nodes of level %d differ in shape", l);
                return HPS_EINVAL;
            }
            for (int t = 0; t < H.n3; ++t) {
                const int ii = iface[J3[t] - op->n_int];
                if (ii < 0) {
                    hps_set_error("internal: merge interface node on the outer boundary");
                    return HPS_EINVAL;
                }
                H.j3i[(size_t)k * H.n3 + t] = ii;
            }
            for (size_t t = 0; t < B.size(); ++t) posB[B[t] - op->n_int] = -1;
            for (int64_t e : J3) in3[e - op->n_int] = 0;
        }
        cur.swap(nxt);
    }
    // root boundary -> boundary index
    root_map.resize(cur[0].size());
    if ((int64_t)cur[0].size() != op->n_bdry) {
        hps_set_error("internal: root boundary size mismatch");
        return HPS_EINVAL;
    }
    for (size_t t = 0; t < cur[0].size(); ++t) {
        const int b = bpos[cur[0][t] - op->n_int];
        if (b < 0) {
            hps_set_error("internal: root boundary node is not on the outer boundary");
            return HPS_EINVAL;
        }
        root_map[t] = b;
    }
    return HPS_OK;
}

// A complex operator is built as the real two-component system of its real embedding.
// Every index set of the scalar tree appears twice (component 0: real part, 1: imaginary
// part).  Leaves order their boundary [component 0 edges | component 1 edges]; an internal
// node orders its boundary [alpha side: component 0, component 1 | beta side: component 0,
// component 1], so that the level kernels' split of a node boundary into its alpha part
// (the first n1 entries) and beta part still holds.  J3 is ordered [component 0 |
// component 1]; interface and boundary data are two planes of the scalar index space.
static void complexify(std::vector<HostLevel> &hl, std::vector<int> &root_map, int q, int64_t n_iface,
                       int64_t n_bdry) {
    const int L = (int)hl.size();
    std::vector<int> sn1(L), sn2(L);
    for (int l = 0; l < L; ++l) {
        sn1[l] = hl[l].n1;
        sn2[l] = hl[l].n2;
    }
    // position of (component c, scalar position t) in a child's two-component boundary
    auto child = [&](int l, int c, int t) -> int {
        if (l == L - 1) return c * 4 * q + t;
        const int n1c = sn1[l + 1], n2c = sn2[l + 1];
        return t < n1c ? c * n1c + t : 2 * n1c + c * n2c + (t - n1c);
    };
    for (int l = 0; l < L; ++l) {
        HostLevel &H = hl[l];
        auto twice = [&](const std::vector<int> &v) {
            std::vector<int> out(2 * v.size());
            for (int c = 0; c < 2; ++c)
                for (size_t k = 0; k < v.size(); ++k) out[c * v.size() + k] = child(l, c, v[k]);
            return out;
        };
        H.a1 = twice(H.a1);
        H.a3 = twice(H.a3);
        H.b2 = twice(H.b2);
        H.b3 = twice(H.b3);
        const size_t nodes = H.n3 ? H.j3i.size() / H.n3 : 0;
        std::vector<int> j3(2 * H.j3i.size());
        for (size_t nd = 0; nd < nodes; ++nd)
            for (int c = 0; c < 2; ++c)
                for (int k = 0; k < H.n3; ++k)
                    j3[nd * 2 * H.n3 + c * H.n3 + k] = (int)(c * n_iface) + H.j3i[nd * H.n3 + k];
        H.j3i.swap(j3);
        H.n1 *= 2;
        H.n2 *= 2;
        H.n3 *= 2;
        H.nbc *= 2;
    }
    std::vector<int> rm(2 * root_map.size());
    if (L == 0) {   // the single leaf's boundary is the root's
        for (int c = 0; c < 2; ++c)
            for (size_t t = 0; t < root_map.size(); ++t) rm[c * root_map.size() + t] = (int)(c * n_bdry) + root_map[t];
    } else {
        const int n1 = sn1[0], n2 = sn2[0];
        for (int c = 0; c < 2; ++c) {
            for (int k = 0; k < n1; ++k) rm[c * n1 + k] = (int)(c * n_bdry) + root_map[k];
            for (int k = 0; k < n2; ++k) rm[2 * n1 + c * n2 + k] = (int)(c * n_bdry) + root_map[n1 + k];
        }
    }
    root_map.swap(rm);
}

// ---------------------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------------------
static int build_impl(hps_op *op, const hps_coeffs *co, const hps_coeffs *co_im, hipStream_t st) {
    const hps_grid &g = op->grid;
    const int m = op->ncomp;
    const int q = op->q, q2 = op->q2 * m, nb4 = 4 * q * m;   // leaf interior / boundary lengths
    const bool ir = (op->flags & HPS_FP32_IR) != 0;
    const bool uni = (op->flags & HPS_UNIFORM_COEFFS) != 0;
    // operators equal at every node of a sweep are packed once (node 0's)
    auto sh = [&](const Panel &p) { return uni ? shared_panel(p) : p; };
    // constants and plan
    std::vector<double> D, D2;
    leaf_derivative(op->p, op->h, D, D2);
    TRY(upload(op, &op->D, D, st));
    TRY(upload(op, &op->D2, D2, st));
    std::vector<int> leaf_ij, root_map, bnd_glob;
    std::vector<HostLevel> hl;
    TRY(plan_tree(op, leaf_ij, hl, root_map, bnd_glob));
    if (m == 2) complexify(hl, root_map, q, op->n_iface, op->n_bdry);
    TRY(upload(op, &op->leaf_ij, leaf_ij, st));
    TRY(upload(op, &op->root_map, root_map, st));
    TRY(upload(op, &op->bnd_glob, bnd_glob, st));
    {
        // boundary index of the two end nodes of every interface line (the line kernel
        // takes them from the boundary data), -1 for lines without unknowns
        std::vector<int> glob_to_b(op->N, -1);
        for (int64_t b = 0; b < op->n_bdry; ++b) glob_to_b[bnd_glob[b]] = (int)b;
        const int nvs = op->grid.n2 * q, nhs = op->grid.n1 * q;
        std::vector<int> ends(2 * (size_t)(nvs + nhs), -1);
        for (int t = 0; t < nvs + nhs; ++t) {
            const bool vert = t < nvs;
            const int n = vert ? op->grid.n1 : op->grid.n2;
            if (n < 2) continue;
            const int line = vert ? t / q : (t - nvs) / q, m0 = (vert ? t : t - nvs) % q;
            const int64_t stride = vert ? (int64_t)op->grid.n2 * q : (int64_t)op->grid.n1 * q;
            const int64_t u0 = vert ? op->n_int + (int64_t)line * q + m0
                                    : op->n_int + op->n_vert + (int64_t)line * q + m0;
            ends[2 * t] = glob_to_b[u0];
            ends[2 * t + 1] = glob_to_b[u0 + n * stride];
        }
        TRY(upload(op, &op->line_ends, ends, st));
    }
    {   // Thomas factors of the interface-line systems (constant coefficients)
        const int nmax = std::max(g.n1, g.n2);
        const double lower = D[(size_t)(op->p - 1) * op->p + 0];
        const double diag = D[(size_t)(op->p - 1) * op->p + (op->p - 1)] - D[0];
        const double upper = -D[op->p - 1];
        op->tri_stride = nmax + 1;
        std::vector<double> tri(2 * (size_t)(nmax + 1), 0.0);
        double cprev = 0.0;
        for (int k = 1; k < nmax; ++k) {
            const double den = diag - (k > 1 ? lower * cprev : 0.0);
            tri[nmax + 1 + k] = 1.0 / den;
            tri[k] = upper / den;
            cprev = tri[k];
        }
        TRY(upload(op, &op->tri_cp, tri, st));
    }
    // coefficients of L (NULL members are zero); complex: real parts, then imaginary parts
    TRY(dev_alloc(op, &op->coef, 5 * m * op->n_int));
    const double *src[10] = {co->cxx, co->cyy, co->cx, co->cy, co->c0, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (co_im) {
        src[5] = co_im->cxx; src[6] = co_im->cyy; src[7] = co_im->cx; src[8] = co_im->cy; src[9] = co_im->c0;
    }
    for (int k = 0; k < 5 * m; ++k) {
        if (src[k])
            HPS_HIP(hipMemcpyAsync(op->coef + k * op->n_int, src[k], sizeof(double) * op->n_int,
                                   hipMemcpyDeviceToDevice, st));
        else
            TRY(launch_zero(op->coef + k * op->n_int, op->n_int, st));
    }
    int *sing;
    TRY(dev_alloc(op, &sing, 1));
    HPS_HIP(hipMemsetAsync(sing, 0, sizeof(int), st));
    if (uni) {   // the caller's claim that the coefficients are constant is checked
        int *diff;
        TRY(dev_alloc(op, &diff, 1));
        HPS_HIP(hipMemsetAsync(diff, 0, sizeof(int), st));
        for (int c = 0; c < m; ++c) TRY(launch_coef_uniform(op->coef + (int64_t)c * 5 * op->n_int, op->n_int, diff, st));
        int hdiff = 0;
        HPS_HIP(hipMemcpyAsync(&hdiff, diff, sizeof(int), hipMemcpyDeviceToHost, st));
        HPS_HIP(hipStreamSynchronize(st));
        CHECK_ARG(hdiff == 0, "HPS_UNIFORM_COEFFS: the coefficients of L vary over the nodes");
    }

    TempBuf tmp(st);
    auto gj_scratch = [&](int n, int nb, unsigned char **used, int **order, double **cb, double **rb) -> int {
        TRY(tmp.get(used, (int64_t)n * nb));
        TRY(tmp.get(order, (int64_t)n * nb));
        TRY(tmp.get(cb, 2 * (int64_t)n * nb));
        TRY(tmp.get(rb, 2 * (int64_t)n * nb));
        return HPS_OK;
    };
    // ---- leaves (Sec. 2.1, eqs. 5-6) ----
    const int nl = op->nleaves;
    // with uniform coefficients every leaf (and every node of a level) has the same
    // operators: compute leaf 0 and node 0 of each level only, the ones the panels keep
    op->build_one = uni;
    const int nlb = uni ? 1 : nl;
    double *W, *Ainv, *S, *T;
    TRY(tmp.get(&W, (int64_t)nlb * q2 * q2));
    TRY(tmp.get(&Ainv, (int64_t)nlb * q2 * q2));
    if (m == 2) TRY(launch_leaf_assemble_cx(op, W, st));
    else TRY(launch_leaf_assemble(op, W, st));
    {
        unsigned char *used; int *order; double *cb, *rb;
        TRY(gj_scratch(q2, nlb, &used, &order, &cb, &rb));
        TRY(gj_invert(W, Ainv, q2, nlb, used, order, cb, rb, sing, st));
        tmp.release(used); tmp.release(order); tmp.release(cb); tmp.release(rb);
    }
    tmp.release(W);
    TRY(tmp.get(&S, (int64_t)nlb * q2 * nb4));
    TRY(tmp.get(&T, (int64_t)nlb * nb4 * nb4));
    if (m == 2) {
        TRY(launch_leaf_S_cx(op, Ainv, S, st));
        TRY(launch_leaf_T_cx(op, S, T, st));
    } else {
        TRY(launch_leaf_S(op, Ainv, S, st));
        TRY(launch_leaf_T(op, S, T, st));
    }
    op->ainv64 = sh(plan_panel(q2, q2, 2, nl, 256, 0));
    op->sleaf64 = sh(plan_panel(q2, nb4, 2, nl, 256, 0));
    for (const Panel *pn : {&op->ainv64, &op->sleaf64})
        if (pn->ntile != 1 || pn->kch != 1) {
            hps_set_error("internal: leaf operator does not fit one workgroup tile");
            return HPS_EINVAL;
        }
    TRY(alloc_panel(op, op->ainv64));
    TRY(alloc_panel(op, op->sleaf64));
    TRY(launch_pack(op->ainv64, Ainv, q2, (int64_t)q2 * q2, q2, nullptr, 0, 0, st));
    TRY(launch_pack(op->sleaf64, S, q2, (int64_t)q2 * nb4, q2, nullptr, 0, 0, st));
    if (ir) {
        op->ainv32 = sh(plan_panel(q2, q2, 4, nl, 256, 0));
        op->sleaf32 = sh(plan_panel(q2, nb4, 4, nl, 256, 0));
        TRY(alloc_panel(op, op->ainv32));
        TRY(alloc_panel(op, op->sleaf32));
        TRY(launch_pack(op->ainv32, Ainv, q2, (int64_t)q2 * q2, q2, nullptr, 0, 0, st,
                        (op->flags & HPS_TEST_FP32_SKEW) ? 1.5 : 1.0));
        TRY(launch_pack(op->sleaf32, S, q2, (int64_t)q2 * nb4, q2, nullptr, 0, 0, st));
    }
    tmp.release(Ainv);
    tmp.release(S);
    TRY(dev_alloc(op, &op->h_leaf, (int64_t)nl * nb4));
    TRY(dev_alloc(op, &op->ub_leaf, (int64_t)nl * nb4));
    TRY(dev_alloc(op, &op->w_leaf, (int64_t)nl * q2));
    TRY(dev_alloc(op, &op->ir_flux, (int64_t)nl * nb4));   // edge flux parts (update, residual)

    // ---- merges, bottom-up (merge formulas after eqs. 7-8) ----
    op->lv.assign(op->L, Level{});
    // level pairs swept through composite operators: the odd level's X, U, S are kept
    // until its parent level (even) has been built, then both are multiplied out
    op->composed = op->composed && compose_eligible(op, hl);
    op->pairs.clear();
    double *kX = nullptr, *kU = nullptr, *kS = nullptr;   // the kept lower level of a pair
    double *Tc = T;
    for (int l = op->L - 1; l >= 0; --l) {
        const HostLevel &H = hl[l];
        Level &Lv = op->lv[l];
        const bool root = (l == 0);
        Lv.nodes = 1 << l;
        Lv.n1 = H.n1; Lv.n2 = H.n2; Lv.n3 = H.n3; Lv.n12 = H.n1 + H.n2; Lv.nbc = H.nbc;
        TRY(upload(op, &Lv.a1, H.a1, st));
        TRY(upload(op, &Lv.a3, H.a3, st));
        TRY(upload(op, &Lv.b2, H.b2, st));
        TRY(upload(op, &Lv.b3, H.b3, st));
        TRY(upload(op, &Lv.j3i, H.j3i, st));
        const int n3 = Lv.n3, n12 = Lv.n12, nbuilt = uni ? 1 : Lv.nodes;   // nodes whose operators are built
        const int64_t s33 = (int64_t)n3 * n3, s3x = (int64_t)n3 * n12, sxx = (int64_t)n12 * n12;
        double *M, *X, *B, *Cm, *Sx, *U, *Tn = nullptr;
        TRY(tmp.get(&M, nbuilt * s33));
        TRY(tmp.get(&X, nbuilt * s33));
        TRY(tmp.get(&B, nbuilt * s3x));
        TRY(tmp.get(&Cm, nbuilt * s3x));
        TRY(tmp.get(&Sx, nbuilt * s3x));
        TRY(tmp.get(&U, nbuilt * s3x));
        if (!root) TRY(tmp.get(&Tn, nbuilt * sxx));
        // children's DtN maps: 2k, 2k+1 of the level below, or the one shared map
        const int64_t cstride = uni ? 0 : (int64_t)Lv.nbc * Lv.nbc;
        TRY(launch_merge_gather(Lv, nbuilt, cstride, root, Tc, M, B, Cm, Tn, st));
        tmp.release(Tc);
        {
            unsigned char *used; int *order; double *cb, *rb;
            TRY(gj_scratch(n3, nbuilt, &used, &order, &cb, &rb));
            TRY(gj_invert(M, X, n3, nbuilt, used, order, cb, rb, sing, st));
            tmp.release(used); tmp.release(order); tmp.release(cb); tmp.release(rb);
        }
        tmp.release(M);
        // S = X [-T^a_31 | T^b_32];  U = [T^a_13; T^b_23] X;  T = diag(T^a_11, T^b_22) + U [...]
        TRY(launch_dgemm(n3, n12, n3, X, n3, s33, B, n3, s3x, Sx, n3, s3x, nbuilt, 1.0, 0.0, st));
        if (!root) {
            TRY(launch_dgemm(n12, n3, n3, Cm, n12, s3x, X, n3, s33, U, n12, s3x, nbuilt, 1.0, 0.0, st));
            TRY(launch_dgemm(n12, n12, n3, U, n12, s3x, B, n3, s3x, Tn, n12, sxx, nbuilt, 1.0, 1.0, st));
        }
        const int rows = root ? n3 : n3 + n12;
        const int rpm = 64, mwg = level_min_wg(op->flags, op->level_mwg);
        Lv.xu64 = sh(plan_panel(rows, n3, 2, Lv.nodes, rpm, mwg));   // tiles planned for every node
        Lv.s64 = sh(plan_panel(n3, n12, 2, Lv.nodes, rpm, mwg));
        TRY(alloc_panel(op, Lv.xu64));
        TRY(alloc_panel(op, Lv.s64));
        TRY(launch_pack(Lv.xu64, X, n3, s33, n3, U, n12, s3x, st));
        TRY(launch_pack(Lv.s64, Sx, n3, s3x, n3, nullptr, 0, 0, st));
        if (ir) {
            Lv.xu32 = sh(plan_panel(rows, n3, 4, Lv.nodes, rpm, mwg));
            Lv.s32 = sh(plan_panel(n3, n12, 4, Lv.nodes, rpm, mwg));
            TRY(alloc_panel(op, Lv.xu32));
            TRY(alloc_panel(op, Lv.s32));
            TRY(launch_pack(Lv.xu32, X, n3, s33, n3, U, n12, s3x, st));
            TRY(launch_pack(Lv.s32, Sx, n3, s3x, n3, nullptr, 0, 0, st));
        }
        tmp.release(B);
        tmp.release(Cm);
        if (op->composed && (l % 2 == 1)) {
            kX = X;   // the lower level of pair (l - 1, l)
            kU = U;
            kS = Sx;
        } else {
            if (op->composed && l + 1 < op->L) {
                TRY(compose_pair(op, l, hl, kX, kU, kS, X, U, Sx, st));
                tmp.release(kX);
                tmp.release(kU);
                tmp.release(kS);
                kX = kU = kS = nullptr;
            }
            tmp.release(X);
            tmp.release(Sx);
            tmp.release(U);
        }
        Tc = Tn;
        // solve workspaces: every node of the level (not only the nodes whose operators were built)
        const int64_t lnodes = Lv.nodes;
        TRY(dev_alloc(op, &Lv.h, lnodes * n12));
        TRY(dev_alloc(op, &Lv.ub, lnodes * n12));
        TRY(dev_alloc(op, &Lv.w3, lnodes * n3));
        int64_t part = 0;
        for (const Panel *pn : {&Lv.xu64, &Lv.s64, &Lv.xu32, &Lv.s32})
            if (pn->kch > 1) part = std::max<int64_t>(part, lnodes * pn->ntile * pn->kch * pn->rp * pn->vw);
        if (part) TRY(dev_alloc(op, &Lv.part, part));
        // split-K arrival counters start at zero; the last arriving workgroup resets them
        int **cnts[4] = {&Lv.cnt_up64, &Lv.cnt_dn64, &Lv.cnt_up32, &Lv.cnt_dn32};
        const Panel *pns[4] = {&Lv.xu64, &Lv.s64, &Lv.xu32, &Lv.s32};
        for (int k = 0; k < 4; ++k) {
            if (pns[k]->kch <= 1) continue;
            const int64_t nc = lnodes * pns[k]->ntile;
            TRY(dev_alloc(op, cnts[k], nc));
            HPS_HIP(hipMemsetAsync(*cnts[k], 0, sizeof(int) * nc, st));
        }
    }
    if (ir) {
        TRY(dev_alloc(op, &op->ir_r, op->n_int));
        TRY(dev_alloc(op, &op->ir_r3, std::max<int64_t>(op->n_iface, 1)));
        TRY(dev_alloc(op, &op->ir_norms, 2));
        TRY(dev_alloc(op, &op->ir_part, 2 * (int64_t)op->nleaves));
        TRY(dev_alloc(op, &op->ir_ubc, 4 * (int64_t)op->q * op->nleaves));
    }
    HPS_HIP(hipStreamSynchronize(st));
    int hsing = 0;
    HPS_HIP(hipMemcpy(&hsing, sing, sizeof(int), hipMemcpyDeviceToHost));
    if (hsing) {
        hps_set_error("a zero pivot occurred while inverting a leaf or merge matrix");
        return HPS_ESINGULAR;
    }
    // the host-side size plan (used to admit operators into a server's cache) must match;
    // composite pairs come on top of it
    std::sort(op->pairs.begin(), op->pairs.end(), [](const PairOps &a, const PairOps &b) { return a.l < b.l; });
    int64_t pair_bytes = 0;
    for (size_t k = 0; k < op->pairs.size(); ++k) {
        if (op->pairs[k].l != 2 * (int)k) {
            hps_set_error("internal: composite pair %zu is for level %d", k, op->pairs[k].l);
            return HPS_EDEVICE;
        }
        pair_bytes += op->pairs[k].up.bytes() + op->pairs[k].dn.bytes() + op->pairs[k].up32.bytes() +
                      op->pairs[k].dn32.bytes();
    }
    if (op->operator_bytes - pair_bytes != plan_operator_bytes(op->grid, op->flags, m, op->level_mwg)) {
        hps_set_error("internal: operator size plan %lld != allocated %lld",
                      (long long)plan_operator_bytes(op->grid, op->flags, m, op->level_mwg),
                      (long long)(op->operator_bytes - pair_bytes));
        return HPS_EDEVICE;
    }
    // small trees: the whole sweep as one product (on top of the plan, like the composites)
    return build_direct(op, st);
}

extern "C" void hps_free(hps_op *op) {
    if (!op) return;
    for (void *p : op->allocs) (void)hipFree(p);
    for (Workspace *w : op->mws) delete w;
    delete op;
}

static int build_op(const hps_grid *grid, const hps_coeffs *coeffs, const hps_coeffs *coeffs_im, double gamma_dt,
                    int flags, void *stream, hps_op **out) {
    CHECK_ARG(out != nullptr, "out is NULL");
    *out = nullptr;
    TRY(check_grid(grid));
    CHECK_ARG(coeffs != nullptr, "coeffs is NULL");
    CHECK_ARG(std::isfinite(gamma_dt) && gamma_dt > 0.0, "gamma_dt must be positive and finite");
    CHECK_ARG((flags & ~(HPS_FP32_IR | HPS_WIDE_TILES | HPS_UNIFORM_COEFFS | HPS_IR_STRICT | HPS_TEST_FP32_SKEW |
                         HPS_AUTOTUNE)) == 0,
              "unknown flags %d", flags);
    CHECK_ARG((flags & HPS_FP32_IR) || !(flags & (HPS_IR_STRICT | HPS_TEST_FP32_SKEW)),
              "flags HPS_IR_STRICT and HPS_TEST_FP32_SKEW apply to HPS_FP32_IR operators only");
    CHECK_ARG(!((flags & HPS_AUTOTUNE) && (flags & HPS_WIDE_TILES)),
              "flags HPS_AUTOTUNE and HPS_WIDE_TILES exclude each other (the tuner times one problem per launch)");
    int mwg = 0, compose = 1;
    if (flags & HPS_AUTOTUNE) {
        flags &= ~HPS_AUTOTUNE;
        TRY(tune_level_tiling(grid, coeffs, coeffs_im, gamma_dt, flags, (hipStream_t)stream, &mwg, &compose));
    }
    return build_op_tiled(grid, coeffs, coeffs_im, gamma_dt, flags, mwg, compose, stream, out);
}

int hps::build_op_tiled(const hps_grid *grid, const hps_coeffs *coeffs, const hps_coeffs *coeffs_im,
                        double gamma_dt, int flags, int mwg, int compose, void *stream, hps_op **out) {
    *out = nullptr;
    const int ncomp = coeffs_im ? 2 : 1;
    if (ncomp == 2) {
        CHECK_ARG(!(flags & HPS_FP32_IR), "complex operators are FP64 only");
        // a leaf's embedded operator (2 (p-2)^2 rows) must fit one workgroup tile
        CHECK_ARG(grid->p <= 18, "complex operators need p <= 18 (got %d)", grid->p);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        hps_set_error("no HIP device is available");
        return HPS_EDEVICE;
    }
    const double *cs[5] = {coeffs->cxx, coeffs->cyy, coeffs->cx, coeffs->cy, coeffs->c0};
    const char *names[5] = {"coeffs.cxx", "coeffs.cyy", "coeffs.cx", "coeffs.cy", "coeffs.c0"};
    for (int k = 0; k < 5; ++k) TRY(check_device_ptr(cs[k], names[k]));
    if (coeffs_im) {
        const double *ci[5] = {coeffs_im->cxx, coeffs_im->cyy, coeffs_im->cx, coeffs_im->cy, coeffs_im->c0};
        for (int k = 0; k < 5; ++k) TRY(check_device_ptr(ci[k], names[k]));
    }
    hps_op *op = new hps_op();
    op->grid = *grid;
    op->p = grid->p;
    op->q = grid->p - 2;
    op->q2 = op->q * op->q;
    op->nleaves = grid->n1 * grid->n2;
    int L = 0;
    while ((1 << L) < op->nleaves) ++L;
    op->L = L;
    const Counts c = counts(grid);
    op->N = c.N; op->n_int = c.n_int; op->n_edge = c.n_edge; op->n_vert = c.n_vert;
    op->n_iface = c.n_iface; op->n_bdry = c.n_bdry;
    op->gamma_dt = gamma_dt;
    op->h = (grid->x1 - grid->x0) / grid->n1;
    op->flags = flags;
    op->ncomp = ncomp;
    op->level_mwg = mwg;
    // composite pair sweeps where the operator allows them (the tuner may choose against
    // them); HPS_COMPOSE=0 turns them off, HPS_COMPOSE=1 on whatever the tuner chose
    const char *cenv = getenv("HPS_COMPOSE");
    op->composed = cenv && cenv[0] ? cenv[0] == '1' : compose != 0;
    int rc;
    {
        HostStage stage((hipStream_t)stream);   // synchronizes and frees at scope exit
        op->stage = &stage;
        rc = build_impl(op, coeffs, coeffs_im, (hipStream_t)stream);
        op->stage = nullptr;
    }
    if (rc) {
        (void)hipDeviceSynchronize();
        hps_free(op);
        return rc;
    }
    *out = op;
    return HPS_OK;
}

extern "C" int hps_build(const hps_grid *grid, const hps_coeffs *coeffs, double gamma_dt, int flags,
                         void *stream, hps_op **out) {
    return build_op(grid, coeffs, nullptr, gamma_dt, flags, stream, out);
}

extern "C" int hps_build_complex(const hps_grid *grid, const hps_coeffs *re, const hps_coeffs *im, double gamma_dt,
                                 int flags, void *stream, hps_op **out) {
    CHECK_ARG(im != nullptr, "im is NULL");
    return build_op(grid, re, im, gamma_dt, flags, stream, out);
}

extern "C" int64_t hps_op_bytes(const hps_op *op, int64_t *operator_bytes) {
    if (!op) {
        hps_set_error("op is NULL");
        return HPS_EINVAL;
    }
    if (operator_bytes) {
        int64_t b = 0;
        const bool f32 = (op->flags & HPS_FP32_IR) != 0;
        b += (f32 ? op->ainv32 : op->ainv64).bytes() + (f32 ? op->sleaf32 : op->sleaf64).bytes();
        if (op->composed) {   // the composites, and the single bottom level of an odd tree
            for (const PairOps &P : op->pairs) b += f32 ? P.up32.bytes() + P.dn32.bytes() : P.up.bytes() + P.dn.bytes();
            if (op->L % 2 == 1) {
                const Level &B = op->lv[op->L - 1];
                b += f32 ? B.xu32.bytes() + B.s32.bytes() : B.xu64.bytes() + B.s64.bytes();
            }
        } else {
            for (const Level &L : op->lv) b += (f32 ? L.xu32 : L.xu64).bytes() + (f32 ? L.s32 : L.s64).bytes();
        }
        *operator_bytes = b;   // bytes streamed by one solve in the op's working precision
    }
    return op->total_bytes;
}

// ---------------------------------------------------------------------------------------
// time stepping
// ---------------------------------------------------------------------------------------
extern "C" int ark_create(hps_op *op, const ark_tableau *tab, double dt, const ark_g *g, ark_ctx **out) {
    CHECK_ARG(out != nullptr, "out is NULL");
    *out = nullptr;
    CHECK_ARG(op != nullptr && tab != nullptr, "op and tab are required");
    CHECK_ARG(tab->s >= 2 && tab->s <= 8, "tableau size s must be in [2, 8]");
    CHECK_ARG(tab->A && tab->b && tab->c && tab->Ahat && tab->bhat, "tableau arrays are required");
    CHECK_ARG(std::isfinite(dt) && dt > 0, "dt must be positive");
    const int s = tab->s;
    CHECK_ARG(tab->A[0] == 0.0, "the ESDIRK tableau must have an explicit first stage");
    const double gam = tab->A[1 * s + 1];
    for (int i = 1; i < s; ++i)
        CHECK_ARG(tab->A[i * s + i] == gam, "the ESDIRK diagonal must be constant (a_ii = gamma)");
    for (int i = 0; i < s; ++i)
        for (int j = i + 1; j < s; ++j)
            CHECK_ARG(tab->A[i * s + j] == 0.0, "the ESDIRK tableau must be lower triangular");
    for (int i = 0; i < s; ++i)
        for (int j = i; j < s; ++j)
            CHECK_ARG(tab->Ahat[i * s + j] == 0.0, "the ERK tableau must be strictly lower triangular");
    CHECK_ARG(std::fabs(gam * dt - op->gamma_dt) <= 1e-14 * op->gamma_dt,
              "operator was built for gamma*dt = %.17g, tableau gives %.17g", op->gamma_dt, gam * dt);
    if (g && op->ncomp == 1) CHECK_ARG(g->kind == 0 || g->kind == 1, "ark_g.kind must be 0 or 1");
    if (g && op->ncomp == 2) CHECK_ARG(g->kind == 0 || g->kind == 2, "a complex operator takes ark_g.kind 0 or 2");
    static std::atomic<uint64_t> next_uid{1};
    ark_ctx *c = new ark_ctx();
    c->uid = next_uid++;
    c->op = op;
    c->s = s;
    c->dt = dt;
    c->A.assign(tab->A, tab->A + s * s);
    c->Ah.assign(tab->Ahat, tab->Ahat + s * s);
    c->b.assign(tab->b, tab->b + s);
    c->bh.assign(tab->bhat, tab->bhat + s);
    c->c.assign(tab->c, tab->c + s);
    if (g) c->g = *g;
    auto fail = [&](int rc) {
        ark_free(c);
        return rc;
    };
    if (int rc = dev_alloc<double>(nullptr, &c->Lu, (int64_t)s * op->ncomp * op->n_int, false)) return fail(rc);
    if (int rc = dev_alloc<double>(nullptr, &c->F, (int64_t)s * op->ncomp * op->n_int, false)) return fail(rc);
    if (int rc = dev_alloc<double>(nullptr, &c->qt_dev, s, false)) return fail(rc);
    if (op->flags & HPS_FP32_IR) {
        if (int rc = dev_alloc<double>(nullptr, &c->rhs, op->n_int, false)) return fail(rc);
        if (int rc = dev_alloc<double>(nullptr, &c->stage_u, op->N, false)) return fail(rc);
        if (int rc = dev_alloc<double>(nullptr, &c->ir_stat, (int64_t)s * IR_MAXIT * 2, false)) return fail(rc);
        if (int rc = dev_alloc<double>(nullptr, &c->u_save, op->N, false)) return fail(rc);
    }
    *out = c;
    return HPS_OK;
}

int64_t hps::ark_ctx_footprint(const hps_op *op, int s) {
    int64_t d = 2LL * s * op->ncomp * op->n_int + s;   // L u_j, F_j, the source's time factors
    if (op->flags & HPS_FP32_IR) d += op->n_int + 2 * op->N + (int64_t)s * IR_MAXIT * 2;
    return 8 * d + workspace_layout(op, nullptr, nullptr, nullptr, nullptr);
}

int hps::ark_slope_workspace(ark_ctx *c) {
    if (c->K) return HPS_OK;
    const hps_op *op = c->op;
    const int64_t s = c->s;
    TRY(dev_alloc<double>(nullptr, &c->K, s * op->N, false));
    TRY(dev_alloc<double>(nullptr, &c->Lk, s * op->n_int, false));
    if (c->g.kind) {
        TRY(dev_alloc<double>(nullptr, &c->Ls, s * op->N, false));
        TRY(dev_alloc<double>(nullptr, &c->Ll, s * op->n_int, false));
    }
    TRY(dev_alloc<double>(nullptr, &c->Lun, op->n_int, false));
    TRY(dev_alloc<double>(nullptr, &c->srhs, op->n_int, false));
    TRY(dev_alloc<double>(nullptr, &c->pen, std::max<int64_t>(op->n_iface, 1), false));
    return HPS_OK;
}

int64_t hps::workspace_layout(const hps_op *op, char *base, Workspace *w, int64_t *cnt_off, int64_t *cnt_bytes) {
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += (std::max<int64_t>(bytes, 8) + 255) & ~int64_t(255);
        return p;
    };
    const int64_t nl = op->nleaves, nb4 = 4 * (int64_t)op->q, q2 = op->q2;
    Workspace tmp;
    Workspace &ws = w ? *w : tmp;
    ws.h_leaf = (double *)take(8 * nl * nb4);
    ws.ub_leaf = (double *)take(8 * nl * nb4);
    ws.w_leaf = (double *)take(8 * nl * q2);
    ws.flux = (double *)take(8 * nl * nb4);
    if (op->flags & HPS_FP32_IR) {
        ws.ir_r = (double *)take(8 * op->n_int);
        ws.ir_r3 = (double *)take(8 * std::max<int64_t>(op->n_iface, 1));
        ws.ir_part = (double *)take(8 * 2 * nl);
        ws.ir_ubc = (double *)take(8 * nl * nb4);
    }
    ws.lv.resize(op->L);
    for (int l = 0; l < op->L; ++l) {
        const Level &L = op->lv[l];
        Workspace::Lv &v = ws.lv[l];
        v = Workspace::Lv{};
        v.h = (double *)take(8 * (int64_t)L.nodes * L.n12);
        v.ub = (double *)take(8 * (int64_t)L.nodes * L.n12);
        v.w3 = (double *)take(8 * (int64_t)L.nodes * L.n3);
        int64_t part = 0;
        for (const Panel *pn : {&L.xu64, &L.s64})
            if (pn->kch > 1) part = std::max<int64_t>(part, (int64_t)L.nodes * pn->ntile * pn->kch * pn->rp * pn->vw);
        if (part) v.part = (double *)take(8 * part);
    }
    // the arrival counters, contiguous at the end
    const int64_t c0 = off;
    for (int l = 0; l < op->L; ++l) {
        const Level &L = op->lv[l];
        Workspace::Lv &v = ws.lv[l];
        if (L.xu64.kch > 1) v.cnt_up = (int *)take(sizeof(int) * (int64_t)L.nodes * L.xu64.ntile);
        if (L.s64.kch > 1) v.cnt_dn = (int *)take(sizeof(int) * (int64_t)L.nodes * L.s64.ntile);
    }
    if (cnt_off) *cnt_off = c0;
    if (cnt_bytes) *cnt_bytes = off - c0;
    return off;
}

// A workspace of the context's own, shaped like its operator's (FP64 levels), in one block.
int hps::ctx_workspace(ark_ctx *c) {
    if (c->ws) return HPS_OK;
    const hps_op *op = c->op;
    int64_t co = 0, cb = 0;
    const int64_t bytes = workspace_layout(op, nullptr, nullptr, &co, &cb);
    void *blk = nullptr;
    if (hipMalloc(&blk, (size_t)bytes) != hipSuccess) {
        hps_set_error("hipMalloc of %lld bytes for a stepping workspace failed", (long long)bytes);
        return HPS_ENOMEM;
    }
    Workspace *w = new Workspace();
    w->allocs.push_back(blk);
    c->ws = w;
    workspace_layout(op, (char *)blk, w, &co, &cb);
    if (cb) HPS_HIP(hipMemset((char *)blk + co, 0, (size_t)cb));
    return HPS_OK;
}

extern "C" void ark_free(ark_ctx *c) {
    if (!c) return;
    if (c->ws) {
        for (void *p : c->ws->allocs) (void)hipFree(p);
        delete c->ws;
    }
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (double *p : {c->Lu, c->F, c->rhs, c->stage_u, c->ir_stat, c->u_save, c->qt_dev, c->K, c->Ls, c->Lk, c->Ll, c->Lun, c->srhs,
                      c->pen})
        if (p) (void)hipFree(p);
    delete c;
}

extern "C" int ark_stage_solves_per_step(const ark_ctx *c) { return c ? c->s - 1 : HPS_EINVAL; }

// ---------------------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------------------
extern "C" int hps_profile_enable(hps_op *op, int enable) {
    CHECK_ARG(op != nullptr, "op is NULL");
    op->prof.on = enable != 0;
    return HPS_OK;
}

extern "C" int hps_profile_read(hps_op *op, int max, const char **names, int64_t *launches, double *total_ms) {
    CHECK_ARG(op != nullptr, "op is NULL");
    CHECK_ARG(max >= 0, "max must be >= 0");
    int64_t cnt[KF_COUNT] = {0};
    double ms[KF_COUNT] = {0};
    for (auto &r : op->prof.recs) {
        HPS_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        HPS_HIP(hipEventElapsedTime(&t, r.a, r.b));
        cnt[r.fam] += 1;
        ms[r.fam] += t;
        op->prof.pool.push_back(r.a);
        op->prof.pool.push_back(r.b);
    }
    op->prof.recs.clear();
    int n = 0;
    for (int f = 0; f < KF_COUNT; ++f) {
        if (!cnt[f]) continue;
        if (n < max) {
            if (names) names[n] = kKernelFamilyNames[f];
            if (launches) launches[n] = cnt[f];
            if (total_ms) total_ms[n] = ms[f];
        }
        ++n;
    }
    return n;
}
