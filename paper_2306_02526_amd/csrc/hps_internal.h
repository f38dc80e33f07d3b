// Internal declarations shared by the HIP kernels and the host side of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "hps.h"

namespace hps {

constexpr int NT = 256;   // threads per workgroup for every kernel of the library
constexpr int PMAX = 24;  // largest supported Chebyshev order p
constexpr int XS_BYTES = 65536;  // LDS bytes for one workgroup's input vector (larger ones are split)

// ---------------------------------------------------------------------------------------
// Packed operator for a streaming matrix-vector product.
//
// A logical R x C matrix (per tree node) is cut into `ntile` row tiles of rp*vw rows and
// `kch` column chunks of S*G columns.  Inside one (tile, chunk) block, thread t = g*rp + r
// of a workgroup owns the vw consecutive rows r*vw .. r*vw+vw-1 of the tile and the
// columns chunk_base + s*G + g, s = 0..S-1.  The block is stored in exactly the order the
// threads read it, [s][t][vw], so every loop iteration of the workgroup reads one
// contiguous run of G*rp 16-byte vectors.  Padding rows/columns hold zeros.
// ---------------------------------------------------------------------------------------
struct Panel {
    int R = 0, C = 0;      // logical shape
    int vw = 2;            // elements per 16-byte vector (2 for FP64, 4 for FP32)
    int rp = 0, G = 0;     // row vectors per tile, column groups
    int ntile = 0, kch = 0, S = 0;
    int64_t tile_elems = 0;   // S*G*rp*vw
    int64_t node_elems = 0;   // ntile*kch*tile_elems
    int nodes = 0;            // nodes stored (1 when shared)
    bool shared = false;      // one copy read by every node of the sweep
    void *data = nullptr;     // double* (vw = 2) or float* (vw = 4)
    int64_t bytes() const { return node_elems * nodes * (vw == 2 ? 8 : 4); }
};

// Choose the packing of an R x C operator for `nodes` nodes.  rp_max bounds the row
// vectors per tile (the leaf kernels need the whole matrix in one tile); min_wg asks
// for at least that many workgroups per sweep (column chunks are added to reach it).
Panel plan_panel(int R, int C, int vw, int nodes, int rp_max, int min_wg);
// The same plan stored once for all `nodes` (operators that are equal at every node).
Panel shared_panel(Panel p);

// what hps_build's panels take (mwg: the tuned minimum of workgroups per level, 0: the rule)
int64_t plan_operator_bytes(const hps_grid &g, int flags, int ncomp = 1, int mwg = 0);
// hps_build's body with a given level tiling (mwg as above; flags without HPS_AUTOTUNE)
int build_op_tiled(const hps_grid *grid, const hps_coeffs *coeffs, const hps_coeffs *coeffs_im, double gamma_dt,
                   int flags, int mwg, int compose, void *stream, hps_op **out);
// composite operators of level pairs (hps_compose.hip)
struct HostLevel;
bool compose_eligible(const hps_op *op, const std::vector<HostLevel> &hl);
int compose_pair(hps_op *op, int l, const std::vector<HostLevel> &hl, const double *Xc, const double *Uc,
                 const double *Sc, const double *Xt, const double *Ut, const double *St, hipStream_t st);
// the direct sweep of a small tree (hps_compose.hip), built after everything else
int build_direct(hps_op *op, hipStream_t st);
int launch_place(double *dst, int ldd, int64_t dstr, int r0, int c0, int rows, int cols, const double *src, int lds,
                 int64_t sstr, const int *ri, const int *cj, double scale, bool accumulate, int batch, hipStream_t st);
// HPS_AUTOTUNE: the level tiling of this operator class, measured on the device the first
// time the class is built (hps_tune.hip)
int tune_level_tiling(const hps_grid *grid, const hps_coeffs *coeffs, const hps_coeffs *coeffs_im, double gamma_dt,
                      int flags, hipStream_t st, int *mwg, int *compose);

// One internal level of the tree (level 0 = root), all nodes of the same shape.
struct Level {
    int nodes = 0;
    int n1 = 0, n2 = 0, n3 = 0, n12 = 0;   // |J1|, |J2|, |J3|, |J1|+|J2|
    int nbc = 0;                            // boundary length of each child (= n1+n3 = n2+n3)
    int *a1 = nullptr, *a3 = nullptr, *b2 = nullptr, *b3 = nullptr;   // device local maps
    int *j3i = nullptr;        // device [nodes][n3]: interface index of each J3 node
    Panel xu64, s64, xu32, s32;
    double *h = nullptr;       // [nodes][n12] particular fluxes (upward sweep)
    double *ub = nullptr;      // [nodes][n12] boundary values (downward sweep)
    double *w3 = nullptr;      // [nodes][n3]
    double *part = nullptr;    // split-K partial sums
    int *cnt_up64 = nullptr, *cnt_dn64 = nullptr, *cnt_up32 = nullptr, *cnt_dn32 = nullptr;  // split-K arrivals
};

// Host copy of one level's index maps (every node of a level has the same local maps):
// node boundary = [alpha's boundary at a1; beta's boundary at b2] (n1 + n2 entries), the
// shared edge J3 at a3 in alpha's boundary and at b3 in beta's; j3i: interface index of
// every J3 node, [nodes][n3].
struct HostLevel {
    int n1 = 0, n2 = 0, n3 = 0, nbc = 0;
    std::vector<int> a1, a3, b2, b3;
    std::vector<int> j3i;   // [nodes][n3]
};

// Two adjacent levels swept by one launch per direction (hps_compose.hip): l is the upper
// level; l = 0 is the top pair (the root and level 1: one launch for both directions).
struct PairOps {
    int l = -1;
    Panel up, dn;                 // composite operators, FP64 (the top pair: dn only)
    Panel up32, dn32;             // FP32 copies (FP32_IR operators)
    int R_up = 0, C_up = 0, R_dn = 0, C_dn = 0;
    int *tab = nullptr;           // device tables
    int t_plus = 0, t_minus = 0, t_j3 = 0, t_fin_up = 0, t_fin_dn = 0, t_copy = 0;
};

// Optional per-kernel timing with HIP events recorded on the launch stream.
enum KernelFamily {
    KF_LEAF_UP64, KF_LEAF_UP32, KF_LEAF_DOWN64, KF_LEAF_DOWN32, KF_LEAF_EVAL_UP64, KF_LEAF_EVAL_UP32,
    KF_LEAF_DOWN_UP64, KF_LEAF_DOWN_UP32, KF_LEAF_DOWN_UPDATE64, KF_LEAF_EVAL_UPDATE64,
    KF_LEVEL_UP64, KF_LEVEL_UP32, KF_LEVEL_DOWN64, KF_LEVEL_DOWN32, KF_RESIDUAL, KF_LINES,
    KF_LEAF2_EVAL_UP64, KF_LEAF2_DOWN_UP64, KF_LEAF2_DOWN_UPDATE64, KF_LEVEL2_UP64, KF_LEVEL2_DOWN64,
    KF_LEAFC_EVAL_UP64, KF_LEAFC_DOWN_UP64, KF_LEAFC_DOWN_UPDATE64, KF_LEAFC_SOLVE64,
    KF_PAIR_UP64, KF_PAIR_TOP64, KF_PAIR_DOWN64, KF_PAIR_UP32, KF_PAIR_TOP32, KF_PAIR_DOWN32, KF_DIRECT64, KF_COUNT
};
extern const char *const kKernelFamilyNames[KF_COUNT];

struct Profiler {
    bool on = false;
    struct Rec {
        int fam;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    ~Profiler();
};

struct ProfScope {
    Profiler *p;
    int fam;
    hipStream_t st;
    hipEvent_t a = nullptr;
    ProfScope(Profiler *p_, int fam_, hipStream_t st_);
    ~ProfScope();
};

// Pinned host staging for the build's host-to-device copies: a copy from pageable memory
// is not asynchronous and waits for the stream to drain, which would leave the GPU idle
// while the host prepares the next level.  copy() puts the data into pinned chunks and
// enqueues the copy on the stream; the destructor synchronizes the stream, then frees the
// chunks.
struct HostStage {
    hipStream_t st = nullptr;
    std::vector<void *> chunks;
    size_t used = 0, cap = 0;
    explicit HostStage(hipStream_t s) : st(s) {}
    HostStage(const HostStage &) = delete;
    HostStage &operator=(const HostStage &) = delete;
    ~HostStage();
    int copy(void *dst, const void *src, size_t bytes);
};

}  // namespace hps

struct hps_op {
    hps_grid grid{};
    int p = 0, q = 0, q2 = 0, L = 0, nleaves = 0;
    int64_t N = 0, n_int = 0, n_edge = 0, n_vert = 0, n_iface = 0, n_bdry = 0;
    double gamma_dt = 0, h = 0;
    int flags = 0;
    // 1: real operator; 2: complex operator stored as its real embedding (every vector in
    // two planes, real part then imaginary part, of the real layout's length)
    int ncomp = 1;
    double *D = nullptr, *D2 = nullptr;    // device p*p, row-major: D[a*p + m] = d/dx weight
    double *coef = nullptr;                // device 5*n_int: cxx, cyy, cx, cy, c0 of L
                                           // (complex: the 5 real parts, then the 5 imaginary)
    int *leaf_ij = nullptr;                // device [nleaves][2] heap order -> (i, j)
    int *root_map = nullptr;               // device [n_bdry] root boundary -> boundary index
    int *bnd_glob = nullptr;               // device [n_bdry] boundary index -> canonical index
    int *line_ends = nullptr;              // device [lines][2] boundary index of each interface
                                           // line's end nodes (-1: a line without unknowns)
    double *tri_cp = nullptr;              // device: Thomas factors cp[k], then 1/den[k]
    int tri_stride = 0;                    // offset of the 1/den table in tri_cp
    hps::Panel ainv64, sleaf64, ainv32, sleaf32;
    std::vector<hps::Level> lv;            // lv[l], l = 0..L-1
    double *h_leaf = nullptr, *ub_leaf = nullptr, *w_leaf = nullptr;
    // HPS_UNIFORM_COEFFS: every leaf, and every node of a level, has the same operators, so
    // the build computes one leaf and one node per level (the panels keep node 0 only)
    bool build_one = false;
    int level_mwg = 0;                     // tuned minimum of workgroups per level (0: the fixed rule)
    // FP64 sweeps of level pairs through composite operators (the per-level operators stay
    // for every other consumer); pairs[k]: upper level 2k (k = 0: the top pair)
    bool composed = false;
    std::vector<hps::PairOps> pairs;
    // small trees: the whole FP64 level sweep without boundary or jump data as one product
    // (build_direct): interface values = M h_leaf, each written to the two leaf-boundary
    // slots it belongs to; the domain-boundary slots get zeros
    bool direct = false;
    hps::Panel dpn;                        // M: [n_iface rows] x [nleaves * 4q columns]
    int *d_rows = nullptr;                 // device [n_iface][2] leaf-boundary slots of each row
    int *d_zero = nullptr;                 // device leaf-boundary slots on the domain boundary
    int n_zero = 0;
    // iterative refinement workspace (FP32_IR)
    double *ir_rhs = nullptr, *ir_r = nullptr, *ir_r3 = nullptr, *ir_du = nullptr, *ir_flux = nullptr;
    double *ir_norms = nullptr;            // [2] max|delta|, max|u| (as ordered bit patterns)
    double *ir_part = nullptr;             // [nleaves][2] per-leaf max|delta|, max|u| of a pass
    double *ir_ubc = nullptr;              // [nleaves][4q] running boundary values of a refined solve
    int64_t operator_bytes = 0, total_bytes = 0;
    std::vector<void *> allocs;
    hps::HostStage *stage = nullptr;   // during the build: staging of host tables
    mutable hps::Profiler prof;
    // solve buffers of right-hand sides 1..3 of a multi-right-hand-side hps_solve (made by
    // its first call; right-hand side 0 uses the operator's own)
    struct Workspace *mws[3] = {nullptr, nullptr, nullptr};
};

// The buffers one FP64 solve writes besides its outputs (leaf boundary values, particular
// solutions and fluxes, per-level boundary data, split-K partials).  An operator owns one
// set; a stepping context gets its own when grouped launches run several contexts of one
// operator together.
struct Workspace {
    struct Lv {
        double *h = nullptr, *ub = nullptr, *w3 = nullptr, *part = nullptr;
        int *cnt_up = nullptr, *cnt_dn = nullptr;
    };
    double *h_leaf = nullptr, *ub_leaf = nullptr, *w_leaf = nullptr, *flux = nullptr;
    double *ir_r = nullptr, *ir_r3 = nullptr;   // FP32_IR operators: the refinement residual
    double *ir_part = nullptr;                  // FP32_IR operators: per-leaf correction norms
    double *ir_ubc = nullptr;                   // FP32_IR operators: running leaf boundary values
    std::vector<Lv> lv;
    std::vector<void *> allocs;
};

namespace hps {
// Layout of one solve's workspace in a single block (256-byte aligned pieces; the split-K
// arrival counters last, at [*cnt_off, *cnt_off + *cnt_bytes), which must hold zeros before
// the first sweep).  Returns the block's size; with base == nullptr only sizes are computed.
int64_t workspace_layout(const hps_op *op, char *base, Workspace *w, int64_t *cnt_off, int64_t *cnt_bytes);
}  // namespace hps

struct ark_ctx {
    hps_op *op = nullptr;
    Workspace *ws = nullptr;              // own workspace for grouped launches (or null)
    uint64_t uid = 0;                     // unique per context created in this process
    int s = 0;
    double dt = 0;
    std::vector<double> A, b, c, Ah, bh;
    ark_g g{};
    double *Lu = nullptr, *F = nullptr;   // device [s][n_int] each
    double *rhs = nullptr;                // device [n_int] (FP32_IR stage right-hand side)
    double *stage_u = nullptr;            // device [N] (FP32_IR stage solution)
    // FP32_IR stage formulation: corrections per stage in the captured step (0 until the
    // first, host-checked step has measured them), the per-stage, per-pass correction
    // norms of a replayed step ([s][IR_MAXIT][2], ordered bits), u^n kept for a redo, and
    // the record of the last step
    int ir_passes = 0;                    // -1: refinement failed for this operator, FP64 stages only
    double *ir_stat = nullptr, *u_save = nullptr;
    hps_info last{};
    double *qt_dev = nullptr;             // device [s]: time factors of a separable source
    // slope formulation (allocated on its first step): slopes k_j [s][N] and l_j [s][N]
    // (l only with g), L k_j and L l_j [s][n_int], L u^n [n_int], the stage right-hand
    // side [n_int] and the penalised flux jumps [n_iface]
    double *K = nullptr, *Ls = nullptr, *Lk = nullptr, *Ll = nullptr, *Lun = nullptr, *srhs = nullptr,
           *pen = nullptr;
    // the FP64 step is replayed from a captured HIP graph while its arguments repeat
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;     // private stream used only for the capture
    std::vector<uintptr_t> gkey;          // array arguments of the captured step
};

// ---------------------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------------------
void hps_set_error(const char *fmt, ...);

#define HPS_HIP(x)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) {                                                                 \
            hps_set_error("%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
            return HPS_EDEVICE;                                                                 \
        }                                                                                       \
    } while (0)

#define HPS_LAUNCHED()  HPS_HIP(hipGetLastError())

#define CHECK_ARG(cond, ...)            \
    do {                                \
        if (!(cond)) {                  \
            hps_set_error(__VA_ARGS__); \
            return HPS_EINVAL;          \
        }                               \
    } while (0)

#define TRY(x)               \
    do {                     \
        int rc_ = (x);       \
        if (rc_) return rc_; \
    } while (0)

// HPS_EINVAL unless p is NULL or a device (or managed) allocation
int check_device_ptr(const void *p, const char *name);

// ---------------------------------------------------------------------------------------
// launchers (hps_solve_kernels.hip, hps_leaf_kernels.hip, hps_build_kernels.hip)
// ---------------------------------------------------------------------------------------
namespace hps {

struct StageCoefs {
    double ca[8];    // dt * a_ij for j < i (ESDIRK)
    double cf[8];    // dt * ahat_ij for j < i (ERK)
    int nprev;       // i (number of previous stages)
};

struct GPoly {
    int kind;
    double g0, g1, g2, g3;
};

// solve sweeps ---------------------------------------------------------------------------
// One per-leaf kernel = a down phase followed by an up phase (hps_leaf_kernels.hip).
enum { LD_NONE = 0, LD_WRITE_U = 1, LD_STAGE = 2, LD_IR_ADD = 3, LD_EVAL = 4 };
enum { LU_NONE = 0, LU_BODY = 1, LU_STAGE = 2, LU_UPDATE = 3 };
struct LeafPhase {
    int down = LD_NONE, up = LU_NONE;
    // down
    const double *u_eval = nullptr;            // LD_EVAL: canonical vector to evaluate
    double *u_out = nullptr;                   // LD_WRITE_U / LD_IR_ADD
    double *Lu_out = nullptr, *F_out = nullptr;  // LD_STAGE / LD_EVAL
    const double *q_src = nullptr;
    double q_scale = 0.0;
    const double *q_scale_ptr = nullptr;   // device scalar; when set it replaces q_scale
    GPoly g{0, 0, 0, 0, 0};
    // up
    const double *body = nullptr;              // LU_BODY
    const double *un = nullptr;                // LU_STAGE / LU_UPDATE
    const double *Lu_in = nullptr, *F_in = nullptr;
    int nprev = 0;                             // stages before the assembled one (newest in LDS)
    double ca[8] = {0}, cf[8] = {0};
    double *rhs_copy = nullptr;
    double *unew = nullptr;                    // LU_UPDATE
    // LD_WRITE_U / LD_IR_ADD with LU_BODY, FP32 operators: the up phase solves for the
    // refinement residual of the u just written, rhs - (I - gamma dt L) u, evaluated in the
    // same kernel (edge fluxes to op->ir_flux for the interface jumps)
    const double *res_rhs = nullptr;
    // LD_IR_ADD with LU_STAGE / LU_UPDATE, FP32 operators: after adding the correction, L u_i
    // and F_i of the corrected u (LD_EVAL's outputs) in the same kernel
    bool ir_eval = false;
    double *norm_part = nullptr;               // LD_IR_ADD: per-leaf max|delta|, max|u| ([leaf][2];
                                               // null: the operator's ir_part), folded by
                                               // launch_norm_fold
};
// ws (FP64 only) redirects the solve buffers (leaf boundary values, particular solutions
// and fluxes) from the operator's own to a workspace
int launch_leaf(const hps_op *op, bool fp32, const LeafPhase &ph, hipStream_t st, const Workspace *ws = nullptr);
// the leaf kernel's down mode for a phase (the LD_ value, or the fused refinement modes:
// residual after LD_WRITE_U / LD_IR_ADD, L u_i and F_i after LD_IR_ADD); grouped launches
// select their kernel with it
int leaf_kernel_mode(const LeafPhase &ph, bool fp32);
// the same phases for a complex operator (FP64; vectors in real / imaginary planes)
int launch_leaf_cx(const hps_op *op, const LeafPhase &ph, hipStream_t st);
// upward sweep over the levels, the root, then the downward sweep (jump and dirichlet
// may be NULL); ws (FP64 only) redirects the per-level buffers to a workspace
int launch_levels(const hps_op *op, bool fp32, const double *jump, const double *dirichlet, hipStream_t st,
                  const Workspace *ws = nullptr);
// step completion after the interior update: boundary data f(t + dt), then the interface
// values from flux continuity along every grid line (reads the leaf edge-flux parts)
int launch_interface_lines(const hps_op *op, double *u, const double *f_end, hipStream_t st,
                           const double *jump = nullptr, const double *fpart = nullptr);
int launch_residual(const hps_op *op, const double *u, const double *rhs, const double *jump,
                    double *r_int, double *r3, hipStream_t st);
int launch_scatter_boundary(const hps_op *op, const double *f, double *u, hipStream_t st);
int launch_zero(double *p, int64_t n, hipStream_t st);
constexpr int kMaxLinComb = 24;
constexpr int IR_MAXIT = 10;          // refinement corrections per solve at most
constexpr double IR_TOL = 1e-11;      // stop when max|delta| <= IR_TOL max|u|
int launch_lincomb(const double *const *v, const double *c, int nv, const double *q, const double *q_scale_ptr,
                   const GPoly *g, double *out, int64_t n, hipStream_t st);
int launch_eval(const hps_op *op, const double *v, double *Lu, bool flux, hipStream_t st);
int launch_flux_jump(const hps_op *op, double scale, double *r3, hipStream_t st);
int ark_slope_workspace(ark_ctx *c);
// device bytes of a stage-formulation context of s stages on op, with its own solve buffers
int64_t ark_ctx_footprint(const hps_op *op, int s);
// the host's part of a refined step that ran a fixed number of corrections per stage
int ir_step_finish(ark_ctx *c, double *u, const double *q_stages, const double *q_space, const double *q_time,
                   const double *f, hipStream_t st, const unsigned long long *stats);
// several operators per launch (FP64 stage formulation): argument records and launches
size_t leaf_args_size();
int fill_leaf_args(const hps_op *op, const LeafPhase &ph, void *dst, size_t *lds, const Workspace *ws,
                   bool fp32 = false);
int ctx_workspace(ark_ctx *c);
int launch_leaf_group(const void *args, const int *base, int nprob, int total, size_t lds, int down, int up,
                      hipStream_t st, bool fp32 = false);
size_t level_record_size();
void level_record(const hps_op *op, int l, bool up, const double *dir, void *dst, int *blocks, size_t *lds,
                  const Workspace *ws, bool fp32 = false, const double *r3 = nullptr);
bool root_fused64(const hps_op *op);
bool root_fused(const hps_op *op, bool fp32);
void root_records(const hps_op *op, const double *dir, void *up_dst, void *dn_dst, int *blocks, size_t *lds,
                  const Workspace *ws, bool fp32 = false, const double *r3 = nullptr);
// refinement residual of several operators: per-problem leaf evaluation records (one
// workgroup per leaf) and interface-jump records (one thread per interface node)
size_t eval_record_size();
size_t jump_record_size();
void residual_records(const hps_op *op, const double *u, const double *rhs, double *r_int, double *r3, double *flux,
                      void *eval_dst, void *jump_dst, int *leaves, int *iface);
int launch_residual_group(const void *evals, const int *ebase, const void *jumps, const int *jbase, int n,
                          int total_leaves, int total_iface, hipStream_t st);
// max|delta| and max|u| of a refinement pass from the per-leaf values the LD_IR_ADD phase
// writes (part[2 leaf], part[2 leaf + 1]) into out[0], out[1] as ordered bit patterns of the
// non-negative doubles; one workgroup per fold, no atomics
struct NormFold {
    const double *part;
    unsigned long long *out;
    int leaves;
};
int launch_norm_fold(const double *part, int leaves, double *out, hipStream_t st);
int launch_norm_fold_group(const NormFold *folds, int n, hipStream_t st);
// copies (src != null) and zero fills of several buffers in one launch
struct MemOp {
    void *dst;
    const void *src;
    int64_t words;   // 8-byte words
};
int launch_memop_group(const MemOp *ops, const int64_t *base, int n, int64_t total, hipStream_t st);
// composite level pairs in grouped launches: mode 0 upward, 1 downward, 2 the top pair
size_t pair_record_size();
int pair_lowest(const hps_op *op);
void pair_record(const hps_op *op, int l, int mode, const double *dir, void *dst, int *blocks, size_t *lds,
                 const Workspace *ws, bool fp32 = false, const double *r3 = nullptr);
int launch_pair_group(const void *args, const int *base, int n, int total, size_t lds, int mode, hipStream_t st,
                      bool fp32 = false);
// the direct product of a small tree (FP64) on the operator's or a workspace's leaf buffers,
// and in grouped launches
int launch_direct(const hps_op *op, hipStream_t st, const Workspace *ws = nullptr);
size_t direct_record_size();
void direct_record(const hps_op *op, void *dst, int *blocks, size_t *lds, const Workspace *ws);
int launch_direct_group(const void *args, const int *base, int n, int total, size_t lds, hipStream_t st);
size_t line_record_size();
void line_record(const hps_op *op, double *u, void *dst, int *systems, const Workspace *ws);
size_t scatter_record_size();
void scatter_record(const hps_op *op, double *u, void *dst, int *count);
int launch_level_group(const void *args, const int *base, int n, int total, size_t lds, bool up, hipStream_t st,
                       bool fp32 = false);
int launch_root_group(const void *ups, const void *dns, const int *base, int n, int total, size_t lds,
                      hipStream_t st, bool fp32 = false);
int launch_lines_group(const void *args, const int *base, int n, int total, hipStream_t st);
int launch_zero_boundary_group(const void *args, const int *base, int n, int total, hipStream_t st);
void step_phase(const ark_ctx *c, int k, double *u, const double *q_stages, const double *q_space,
                const double *qt, LeafPhase &ph);
// two components on one operator (FP64): both components' leaf phase in one launch, and
// the level sweeps of both (ws[c]: component c's solve buffers, null for the operator's)
int launch_leaf_sys(const hps_op *op, const LeafPhase &ph0, const LeafPhase &ph1, const Workspace *ws0,
                    const Workspace *ws1, hipStream_t st);
int launch_levels_sys(const hps_op *op, const Workspace *const ws[2], const double *const dir[2], hipStream_t st);
int launch_set_values(double *dst, const double *vals, int n, hipStream_t st);   // n <= 8, vals on the host
// nc = 2..4 right-hand sides of one FP64 operator per launch (hps_solve with nrhs > 1):
// the leaf particular solves (up) or reconstructions (down) and the level sweeps; ws[c]:
// right-hand side c's solve buffers (null: the operator's own)
constexpr int MAX_MULTI = 4;
int launch_leaf_multi(const hps_op *op, int nc, bool up, const double *const *body, double *const *u,
                      const Workspace *const *ws, hipStream_t st);
int launch_levels_multi(const hps_op *op, int nc, const Workspace *const *ws, const double *const *dir,
                        const double *const *jump, hipStream_t st);
bool levels_multi_fit(const hps_op *op, int nc);   // the level products' LDS for nc right-hand sides fits

// build --------------------------------------------------------------------------------
int launch_leaf_assemble(const hps_op *op, double *W, hipStream_t st);
// complex operators: the real embeddings [[Re, -Im], [Im, Re]] of A_ii, S_leaf and the DtN map
int launch_leaf_assemble_cx(const hps_op *op, double *W, hipStream_t st);
int launch_leaf_S_cx(const hps_op *op, const double *ainv, double *S, hipStream_t st);
int launch_leaf_T_cx(const hps_op *op, const double *S, double *T, hipStream_t st);
// sets *flag (device int, zero beforehand) when some coefficient differs from its value at
// node 0
int launch_coef_uniform(const double *coef, int64_t n, int *flag, hipStream_t st);
// out = inverse of each of the nb n x n matrices in W (column-major, partial pivoting; W is
// overwritten, out serves as the second copy of the batch while the pivot steps run);
// scratch: used [n nb] bytes, order [n nb], colbuf and rowbuf [2 n nb] each; *sing is set
// when a pivot is zero or not finite
int gj_invert(double *W, double *out, int n, int nb, unsigned char *used, int *order,
              double *colbuf, double *rowbuf, int *sing, hipStream_t st);
int launch_leaf_S(const hps_op *op, const double *ainv, double *S, hipStream_t st);
int launch_leaf_T(const hps_op *op, const double *S, double *T, hipStream_t st);
int launch_merge_gather(const Level &L, int nodes, int64_t child_stride, bool root, const double *Tc, double *M, double *B,
                        double *Cm, double *Tn, hipStream_t st);
int launch_dgemm(int M, int N, int K, const double *A, int lda, int64_t sA, const double *B,
                 int ldb, int64_t sB, double *C, int ldc, int64_t sC, int batch, double alpha,
                 double beta, hipStream_t st);
// Pack a column-major operator (rows [0,rows0) from src0, rows [rows0,R) from src1) into a
// Panel, as FP64 or FP32 according to pn.vw.
int launch_pack(const Panel &pn, const double *src0, int ld0, int64_t stride0, int rows0,
                const double *src1, int ld1, int64_t stride1, hipStream_t st, double scale = 1.0);
int launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);

}  // namespace hps
