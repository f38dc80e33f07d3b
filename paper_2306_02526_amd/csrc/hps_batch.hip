// Batched entry points: many independent problems per call.  Time steps of FP64 problems,
// and refined steps of FP32_IR problems after their first step, run as grouped launches
// (one launch per leaf phase and per tree level for all problems of a kind and stage
// count); everything else runs each problem through the single-problem entry points on a
// pool of library-owned HIP streams, so that small problems overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "hps_batch.h"
#include "hps_internal.h"

using namespace hps;

namespace {

// Four streams: the number of hardware queues HIP gives a process by default, so each
// stream gets its own queue and the problems on different streams run concurrently.
constexpr int kStreams = 4;

struct StreamPool {
    hipStream_t s[kStreams] = {};
    hipEvent_t done[kStreams] = {};
    hipEvent_t fork = nullptr;
    std::mutex busy;   // one batched call per device at a time (the events are reused)
};

std::mutex g_pools_mu;
std::map<int, StreamPool *> g_pools;   // per device; kept until the process ends

int pool_for_current_device(StreamPool **out) {
    int dev = 0;
    HPS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_pools_mu);
    auto it = g_pools.find(dev);
    if (it != g_pools.end()) {
        *out = it->second;
        return HPS_OK;
    }
    StreamPool *p = new StreamPool;
    for (int k = 0; k < kStreams; ++k) {
        HPS_HIP(hipStreamCreateWithFlags(&p->s[k], hipStreamNonBlocking));
        HPS_HIP(hipEventCreateWithFlags(&p->done[k], hipEventDisableTiming));
    }
    HPS_HIP(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    g_pools[dev] = p;
    *out = p;
    return HPS_OK;
}

// Longest-processing-time assignment: problems by decreasing operator bytes (the bytes
// one solve streams), each onto the stream with the least bytes so far; problems that
// share an operator follow the stream of its first problem.
std::vector<int> assign_streams(const std::vector<const hps_op *> &ops) {
    const int n = (int)ops.size();
    std::vector<int> order(n), lane(n, -1);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return ops[a]->operator_bytes > ops[b]->operator_bytes;
    });
    std::map<const hps_op *, int> owner;
    double load[kStreams] = {};
    for (int b : order) {
        auto it = owner.find(ops[b]);
        int k;
        if (it != owner.end()) {
            k = it->second;
        } else {
            k = (int)(std::min_element(load, load + kStreams) - load);
            owner[ops[b]] = k;
        }
        lane[b] = k;
        load[k] += (double)ops[b]->operator_bytes;
    }
    return lane;
}

int tag_problem(int rc, int b) {
    std::string msg = hps_last_error();
    hps_set_error("problem %d: %s", b, msg.c_str());
    return rc;
}

// Runs fn(b, stream) for every problem on its assigned pool stream, in batch order per
// stream, between a fork from and a join back to the caller's stream.
template <class Fn>
int run_batched(const std::vector<const hps_op *> &ops, hipStream_t caller, Fn fn,
                const std::vector<int> *ids = nullptr) {
    StreamPool *pool = nullptr;
    TRY(pool_for_current_device(&pool));
    std::lock_guard<std::mutex> g(pool->busy);
    const std::vector<int> lane = assign_streams(ops);
    bool used[kStreams] = {};
    for (int k : lane) used[k] = true;
    HPS_HIP(hipEventRecord(pool->fork, caller));
    for (int k = 0; k < kStreams; ++k)
        if (used[k]) HPS_HIP(hipStreamWaitEvent(pool->s[k], pool->fork, 0));
    int rc = HPS_OK;
    for (int b = 0; b < (int)ops.size() && rc == HPS_OK; ++b) {
        rc = fn(b, pool->s[lane[b]]);
        if (rc != HPS_OK) rc = tag_problem(rc, ids ? (*ids)[b] : b);   // the caller's problem index
    }
    // join even after an error, so the caller's stream still orders after what ran
    for (int k = 0; k < kStreams; ++k) {
        if (!used[k]) continue;
        HPS_HIP(hipEventRecord(pool->done[k], pool->s[k]));
        HPS_HIP(hipStreamWaitEvent(caller, pool->done[k], 0));
    }
    return rc;
}

// ---- all problems of a batch in one launch per phase (FP64 stage formulation) ----------
// One launch runs a leaf phase for the leaves of every problem, one launch a tree level
// (levels aligned at the roots), one the fused roots, one the line solves: a step of any
// number of problems takes as many launches as a step of the largest one.  The argument
// records live in device memory, built once per set of (context, u, source) pointers,
// and the step is captured into a HIP graph and replayed while that set repeats.
// An event shared by a retired plan and its pooled blocks, destroyed with its last holder.
struct SharedEvent {
    hipEvent_t e = nullptr;
    int refs = 0;
};

void unref(SharedEvent *ev) {
    if (ev && --ev->refs == 0) {
        if (ev->e) (void)hipEventDestroy(ev->e);
        delete ev;
    }
}

struct GroupPlan {
    struct Launch {
        int kind;            // 0 leaf phase, 1 level up, 2 level down, 3 roots, 4 boundary, 5 lines,
                             // 6 / 7 / 8 composite pairs up / down / top, 9 copies and fills,
                             // 10 refinement residuals, 11 correction-norm folds, 12 direct
                             // products of small trees
        size_t a, a2, base;  // offsets of the records (a2: downward root records / jump
                             // records) and bases
        int cnt, total;
        size_t lds;
        int down, up;
        int fp32 = 0;        // FP32 operators (refined steps)
        size_t base2 = 0;    // residuals: bases of the jump records
        int total2 = 0;      // residuals: interface nodes; copies and fills: words (low 31 bits
        int64_t words = 0;   // unused otherwise)
    };
    bool ir = false;                     // refined FP32 steps: `seq` in order
    std::vector<Launch> seq;
    std::vector<uintptr_t> key;
    int s = 0, n = 0;
    unsigned char *dmem = nullptr;       // the records (a block of the pool)
    size_t dbytes = 0;
    unsigned char *qblk = nullptr;       // the separable sources' time factors (a pool block)
    size_t qbytes = 0;
    double *qt = nullptr;                // = qblk: device [n][8]
    std::vector<unsigned char> host;     // host copy of the records (read by the upload)
    std::vector<Launch> leaf, sweep;
    Launch zb{}, lines{};
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    SharedEvent *done = nullptr;         // recorded after every launch of the plan
    int uses = 0;
    uint64_t last_use = 0;
};

// Plans are cheap to replace: a new set of problems (every arrival or completion in a
// server) takes its device blocks from a pool instead of hipMalloc (and an evicted plan's
// blocks go back to it instead of hipFree, which would wait for the whole device); the
// records are uploaded asynchronously behind the block's previous use; the first step of
// a set runs without a graph (capture and instantiation pay off only for a set that
// repeats); an evicted plan's graph is destroyed once its last launch has completed.
std::mutex g_plans_mu;
std::vector<GroupPlan *> g_plans;   // a few recent plans (each set of problems has one)
uint64_t g_plan_clock = 0;
constexpr size_t kMaxPlans = 4;

struct PoolBlock {
    unsigned char *p;
    size_t bytes;
    SharedEvent *last;   // completion of the block's last use (null if none)
};
std::vector<PoolBlock> g_blocks;    // free device blocks
std::vector<GroupPlan *> g_retired; // evicted plans whose last launch may still run

// A device block of at least `bytes`, usable on stream st (st first waits for its last use).
int take_block(size_t bytes, hipStream_t st, unsigned char **out, size_t *got) {
    size_t best = g_blocks.size();
    for (size_t k = 0; k < g_blocks.size(); ++k)
        if (g_blocks[k].bytes >= bytes && (best == g_blocks.size() || g_blocks[k].bytes < g_blocks[best].bytes))
            best = k;
    if (best < g_blocks.size()) {
        PoolBlock b = g_blocks[best];
        g_blocks.erase(g_blocks.begin() + (long)best);
        hipError_t e = hipSuccess;
        if (b.last) e = hipStreamWaitEvent(st, b.last->e, 0);
        unref(b.last);
        *out = b.p;
        *got = b.bytes;
        HPS_HIP(e);
        return HPS_OK;
    }
    const size_t sz = std::max<size_t>((bytes + 65535) & ~size_t(65535), 65536);
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        hps_set_error("hipMalloc of %zu bytes for grouped-launch records failed", sz);
        return HPS_ENOMEM;
    }
    *out = (unsigned char *)p;
    *got = sz;
    return HPS_OK;
}

void destroy_plan_objects(GroupPlan *p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    unref(p->done);
    delete p;
}

// Retire an evicted (or failed) plan: its blocks go back to the pool, each holding the
// plan's completion event; the plan waits in g_retired until its last launch is done.
void retire_plan(GroupPlan *p) {
    SharedEvent *ev = p->uses > 0 ? p->done : nullptr;
    for (auto blk : {std::make_pair(p->dmem, p->dbytes), std::make_pair(p->qblk, p->qbytes)}) {
        if (!blk.first) continue;
        if (ev) ev->refs++;
        g_blocks.push_back(PoolBlock{blk.first, blk.second, ev});
    }
    p->dmem = p->qblk = nullptr;
    g_retired.push_back(p);
}

// Destroy the retired plans whose last launch has completed (never waits).
void reap_retired() {
    for (size_t k = 0; k < g_retired.size();) {
        GroupPlan *p = g_retired[k];
        const bool busy = p->uses > 0 && p->done && hipEventQuery(p->done->e) != hipSuccess;
        if (busy) {
            (void)hipGetLastError();   // not ready is not an error here
            ++k;
            continue;
        }
        destroy_plan_objects(p);
        g_retired.erase(g_retired.begin() + (long)k);
    }
}

struct HostTables {
    std::vector<unsigned char> bytes;
    size_t put(const void *src, size_t n) {
        const size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + n);
        if (src) std::memcpy(bytes.data() + off, src, n);
        return off;
    }
};

bool groupable(ark_ctx *const *ctx, int nprob, const double *const *q_stages, const double *const *f_stages) {
    const char *env = getenv("HPS_GROUP");
    if (env && env[0] == '0') return false;
    for (int b = 0; b < nprob; ++b) {
        const hps_op *op = ctx[b]->op;
        if ((op->flags & HPS_FP32_IR) || op->ncomp != 1) return false;
        if (op->prof.on || op->L < 1 || ctx[b]->s != ctx[0]->s) return false;
        if (f_stages && f_stages[b]) return false;
    }
    (void)q_stages;
    return true;
}

int build_plan(GroupPlan *P, ark_ctx *const *ctx, int n, double *const *u, const double *const *q_stages,
               const double *const *q_space, hipStream_t st) {
    P->n = n;
    P->s = ctx[0]->s;
    // problems that share an operator each write a workspace of their own
    std::map<const hps_op *, int> uses;
    for (int b = 0; b < n; ++b) uses[ctx[b]->op]++;
    std::vector<const Workspace *> ws(n, nullptr);
    for (int b = 0; b < n; ++b)
        if (uses[ctx[b]->op] > 1) {
            TRY(ctx_workspace(ctx[b]));
            ws[b] = ctx[b]->ws;
        }
    TRY(take_block(sizeof(double) * 8 * n, st, &P->qblk, &P->qbytes));
    P->qt = reinterpret_cast<double *>(P->qblk);
    TRY(launch_zero(P->qt, 8 * (int64_t)n, st));
    HostTables T;
    std::vector<int> base(n + 1);
    // leaf phases
    for (int k = 0; k < P->s; ++k) {
        GroupPlan::Launch L{};
        L.kind = 0;
        const size_t rs = leaf_args_size();
        std::vector<unsigned char> recs(rs * n);
        base[0] = 0;
        for (int b = 0; b < n; ++b) {
            LeafPhase ph;
            step_phase(ctx[b], k, u[b], q_stages ? q_stages[b] : nullptr, q_space ? q_space[b] : nullptr,
                       P->qt + 8 * b, ph);
            size_t lds = 0;
            TRY(fill_leaf_args(ctx[b]->op, ph, recs.data() + rs * b, &lds, ws[b]));
            L.lds = std::max(L.lds, lds);
            L.down = ph.down;
            L.up = ph.up;
            base[b + 1] = base[b] + ctx[b]->op->nleaves;
        }
        L.a = T.put(recs.data(), recs.size());
        L.base = T.put(base.data(), sizeof(int) * (n + 1));
        L.cnt = n;
        L.total = base[n];
        P->leaf.push_back(L);
    }
    // one sweep: upward levels aligned at the roots, the fused roots, downward levels
    int Lmax = 0;
    for (int b = 0; b < n; ++b) Lmax = std::max(Lmax, ctx[b]->op->L);
    const size_t ls = level_record_size(), prs = pair_record_size();
    // operators with composite level pairs sweep pair (l, l + 1) at its upper level l and
    // only the bottom level of an odd tree with the single-level kernels
    // small trees with a direct product sweep in one launch of their own, as a single step does
    auto single_here = [&](const hps_op *op, int l) -> bool {
        if (l >= op->L || op->direct) return false;
        if (op->composed) return (op->L % 2 == 1) && l == op->L - 1;
        return !(l == 0 && root_fused64(op));
    };
    auto pair_here = [&](const hps_op *op, int l, int mode) -> bool {
        if (!op->composed || op->direct) return false;
        if (mode == 2) return l == 0;
        return l >= 2 && l % 2 == 0 && l <= pair_lowest(op);
    };
    auto pair_launch = [&](int l, int mode) -> int {   // mode 0 up, 1 down, 2 the top pairs
        GroupPlan::Launch L{};
        L.kind = 6 + mode;
        std::vector<unsigned char> recs;
        std::vector<int> bs(1, 0);
        for (int b = 0; b < n; ++b) {
            const hps_op *op = ctx[b]->op;
            if (!pair_here(op, l, mode)) continue;
            recs.resize(recs.size() + prs);
            int blocks = 0;
            size_t lds = 0;
            pair_record(op, l, mode, nullptr, recs.data() + recs.size() - prs, &blocks, &lds, ws[b]);
            L.lds = std::max(L.lds, lds);
            bs.push_back(bs.back() + blocks);
        }
        L.cnt = (int)bs.size() - 1;
        if (L.cnt == 0) return HPS_OK;
        L.a = T.put(recs.data(), recs.size());
        L.base = T.put(bs.data(), sizeof(int) * bs.size());
        L.total = bs.back();
        P->sweep.push_back(L);
        return HPS_OK;
    };
    auto level_launch = [&](int l, bool up) -> int {
        GroupPlan::Launch L{};
        L.kind = up ? 1 : 2;
        std::vector<unsigned char> recs;
        std::vector<int> bs(1, 0);
        for (int b = 0; b < n; ++b) {
            const hps_op *op = ctx[b]->op;
            if (!single_here(op, l)) continue;
            recs.resize(recs.size() + ls);
            int blocks = 0;
            size_t lds = 0;
            level_record(op, l, up, nullptr, recs.data() + recs.size() - ls, &blocks, &lds, ws[b]);
            L.lds = std::max(L.lds, lds);
            bs.push_back(bs.back() + blocks);
        }
        L.cnt = (int)bs.size() - 1;
        if (L.cnt == 0) return HPS_OK;
        L.a = T.put(recs.data(), recs.size());
        L.base = T.put(bs.data(), sizeof(int) * bs.size());
        L.total = bs.back();
        P->sweep.push_back(L);
        return HPS_OK;
    };
    {
        GroupPlan::Launch L{};
        L.kind = 12;
        const size_t ds = direct_record_size();
        std::vector<unsigned char> recs;
        std::vector<int> bs(1, 0);
        for (int b = 0; b < n; ++b) {
            const hps_op *op = ctx[b]->op;
            if (!op->direct) continue;
            recs.resize(recs.size() + ds);
            int blocks = 0;
            size_t lds = 0;
            direct_record(op, recs.data() + recs.size() - ds, &blocks, &lds, ws[b]);
            L.lds = std::max(L.lds, lds);
            bs.push_back(bs.back() + blocks);
        }
        L.cnt = (int)bs.size() - 1;
        if (L.cnt > 0) {
            L.a = T.put(recs.data(), recs.size());
            L.base = T.put(bs.data(), sizeof(int) * bs.size());
            L.total = bs.back();
            P->sweep.push_back(L);
        }
    }
    for (int l = Lmax - 1; l >= 0; --l) {
        TRY(level_launch(l, true));
        TRY(pair_launch(l, 0));
    }
    TRY(pair_launch(0, 2));
    {
        GroupPlan::Launch L{};
        L.kind = 3;
        std::vector<unsigned char> ups, dns;
        std::vector<int> bs(1, 0);
        for (int b = 0; b < n; ++b) {
            const hps_op *op = ctx[b]->op;
            if (op->composed || op->direct || !root_fused64(op)) continue;
            ups.resize(ups.size() + ls);
            dns.resize(dns.size() + ls);
            int blocks = 0;
            size_t lds = 0;
            root_records(op, nullptr, ups.data() + ups.size() - ls, dns.data() + dns.size() - ls, &blocks, &lds, ws[b]);
            L.lds = std::max(L.lds, lds);
            bs.push_back(bs.back() + blocks);
        }
        L.cnt = (int)bs.size() - 1;
        if (L.cnt > 0) {
            L.a = T.put(ups.data(), ups.size());
            L.a2 = T.put(dns.data(), dns.size());
            L.base = T.put(bs.data(), sizeof(int) * bs.size());
            L.total = bs.back();
            P->sweep.push_back(L);
        }
    }
    for (int l = 0; l < Lmax; ++l) {
        TRY(pair_launch(l, 1));
        TRY(level_launch(l, false));
    }
    // boundary values (zero) and interface line solves of the update
    {
        const size_t zs = scatter_record_size(), lr = line_record_size();
        std::vector<unsigned char> zrec(zs * n), lrec(lr * n);
        std::vector<int> zb(n + 1, 0), lb(n + 1, 0);
        for (int b = 0; b < n; ++b) {
            int cnt = 0, sys = 0;
            scatter_record(ctx[b]->op, u[b], zrec.data() + zs * b, &cnt);
            line_record(ctx[b]->op, u[b], lrec.data() + lr * b, &sys, ws[b]);
            zb[b + 1] = zb[b] + cnt;
            lb[b + 1] = lb[b] + sys;
        }
        P->zb = GroupPlan::Launch{4, T.put(zrec.data(), zrec.size()), 0, T.put(zb.data(), sizeof(int) * (n + 1)),
                                  n, zb[n], 0, 0, 0};
        P->lines = GroupPlan::Launch{5, T.put(lrec.data(), lrec.size()), 0, T.put(lb.data(), sizeof(int) * (n + 1)),
                                     n, lb[n], 0, 0, 0};
    }
    P->host.swap(T.bytes);
    TRY(take_block(std::max<size_t>(P->host.size(), 256), st, &P->dmem, &P->dbytes));
    HPS_HIP(hipMemcpyAsync(P->dmem, P->host.data(), P->host.size(), hipMemcpyHostToDevice, st));
    P->done = new SharedEvent();
    P->done->refs = 1;
    HPS_HIP(hipEventCreateWithFlags(&P->done->e, hipEventDisableTiming));
    return HPS_OK;
}

// Refined FP32 steps of several problems (FP32_IR operators whose contexts have made their
// first, host-checked step): the launches of enqueue_step's fixed-pass refinement for all
// problems at once -- each problem keeps its own number of passes (a pass's launches cover
// the problems that still have that pass), so every problem runs exactly the kernels and
// arithmetic of its single step.
bool groupable_ir(ark_ctx *const *ctx, int nprob, const double *const *f_stages) {
    const char *env = getenv("HPS_GROUP");
    if (env && env[0] == '0') return false;
    for (int b = 0; b < nprob; ++b) {
        const hps_op *op = ctx[b]->op;
        if (!(op->flags & HPS_FP32_IR) || op->ncomp != 1 || op->prof.on || op->L < 1) return false;
        if (ctx[b]->s != ctx[0]->s || ctx[b]->ir_passes <= 0) return false;
        if (f_stages && f_stages[b]) return false;
        for (const Level &lv : op->lv)
            if (lv.xu32.kch != 1 || lv.s32.kch != 1) return false;
    }
    return true;
}

int build_plan_ir(GroupPlan *P, ark_ctx *const *ctx, int n, double *const *u, const double *const *q_stages,
                  const double *const *q_space, hipStream_t st) {
    P->n = n;
    P->s = ctx[0]->s;
    P->ir = true;
    const int s = P->s;
    std::map<const hps_op *, int> uses;
    for (int b = 0; b < n; ++b) uses[ctx[b]->op]++;
    std::vector<const Workspace *> ws(n, nullptr);
    for (int b = 0; b < n; ++b)
        if (uses[ctx[b]->op] > 1) {
            TRY(ctx_workspace(ctx[b]));
            ws[b] = ctx[b]->ws;
        }
    TRY(take_block(sizeof(double) * 8 * n, st, &P->qblk, &P->qbytes));
    P->qt = reinterpret_cast<double *>(P->qblk);
    TRY(launch_zero(P->qt, 8 * (int64_t)n, st));
    HostTables T;
    std::vector<int> all(n);
    std::iota(all.begin(), all.end(), 0);
    auto r_of = [&](int b) { return ws[b] ? ws[b]->ir_r : ctx[b]->op->ir_r; };
    auto r3_of = [&](int b) -> double * {
        if (!ctx[b]->op->n_iface) return nullptr;
        return ws[b] ? ws[b]->ir_r3 : ctx[b]->op->ir_r3;
    };
    auto flux_of = [&](int b) { return ws[b] ? ws[b]->flux : ctx[b]->op->ir_flux; };
    auto part_of = [&](int b) { return ws[b] ? ws[b]->ir_part : ctx[b]->op->ir_part; };
    // one leaf phase (the same kinds for all listed problems)
    auto leaf = [&](const std::vector<int> &probs, auto phase) -> int {
        GroupPlan::Launch L{};
        L.kind = 0;
        L.fp32 = 1;
        const size_t rs = leaf_args_size();
        std::vector<unsigned char> recs(rs * probs.size());
        std::vector<int> base(probs.size() + 1, 0);
        for (size_t i = 0; i < probs.size(); ++i) {
            const int b = probs[i];
            LeafPhase ph;
            phase(b, ph);
            size_t lds = 0;
            TRY(fill_leaf_args(ctx[b]->op, ph, recs.data() + rs * i, &lds, ws[b], true));
            L.lds = std::max(L.lds, lds);
            L.down = leaf_kernel_mode(ph, true);
            L.up = ph.up;
            base[i + 1] = base[i] + ctx[b]->op->nleaves;
        }
        L.a = T.put(recs.data(), recs.size());
        L.base = T.put(base.data(), sizeof(int) * base.size());
        L.cnt = (int)probs.size();
        L.total = base.back();
        P->seq.push_back(L);
        return HPS_OK;
    };
    // the FP32 level sweeps (upward levels aligned at the roots, the fused roots and top
    // pairs, downward); operators with composite pairs take them at the pair's upper level
    const size_t ls = level_record_size(), prs = pair_record_size();
    auto single_here = [&](const hps_op *op, int l) -> bool {
        if (l >= op->L) return false;
        if (op->composed) return (op->L % 2 == 1) && l == op->L - 1;
        return !(l == 0 && root_fused(op, true));
    };
    auto pair_here = [&](const hps_op *op, int l, int mode) -> bool {
        if (!op->composed) return false;
        if (mode == 2) return l == 0;
        return l >= 2 && l % 2 == 0 && l <= pair_lowest(op);
    };
    auto sweep = [&](const std::vector<int> &probs, bool with_r3) -> int {
        int Lmax = 0;
        for (int b : probs) Lmax = std::max(Lmax, ctx[b]->op->L);
        auto pairs = [&](int l, int mode) -> int {
            GroupPlan::Launch L{};
            L.kind = 6 + mode;
            L.fp32 = 1;
            std::vector<unsigned char> recs;
            std::vector<int> bs(1, 0);
            for (int b : probs) {
                const hps_op *op = ctx[b]->op;
                if (!pair_here(op, l, mode)) continue;
                recs.resize(recs.size() + prs);
                int blocks = 0;
                size_t lds = 0;
                pair_record(op, l, mode, nullptr, recs.data() + recs.size() - prs, &blocks, &lds, ws[b], true,
                            with_r3 ? r3_of(b) : nullptr);
                L.lds = std::max(L.lds, lds);
                bs.push_back(bs.back() + blocks);
            }
            L.cnt = (int)bs.size() - 1;
            if (L.cnt == 0) return HPS_OK;
            L.a = T.put(recs.data(), recs.size());
            L.base = T.put(bs.data(), sizeof(int) * bs.size());
            L.total = bs.back();
            P->seq.push_back(L);
            return HPS_OK;
        };
        auto level = [&](int l, bool up) -> int {
            GroupPlan::Launch L{};
            L.kind = up ? 1 : 2;
            L.fp32 = 1;
            std::vector<unsigned char> recs;
            std::vector<int> bs(1, 0);
            for (int b : probs) {
                const hps_op *op = ctx[b]->op;
                if (!single_here(op, l)) continue;
                recs.resize(recs.size() + ls);
                int blocks = 0;
                size_t lds = 0;
                level_record(op, l, up, nullptr, recs.data() + recs.size() - ls, &blocks, &lds, ws[b], true,
                             with_r3 ? r3_of(b) : nullptr);
                L.lds = std::max(L.lds, lds);
                bs.push_back(bs.back() + blocks);
            }
            L.cnt = (int)bs.size() - 1;
            if (L.cnt == 0) return HPS_OK;
            L.a = T.put(recs.data(), recs.size());
            L.base = T.put(bs.data(), sizeof(int) * bs.size());
            L.total = bs.back();
            P->seq.push_back(L);
            return HPS_OK;
        };
        for (int l = Lmax - 1; l >= 0; --l) {
            TRY(level(l, true));
            TRY(pairs(l, 0));
        }
        TRY(pairs(0, 2));
        {
            GroupPlan::Launch L{};
            L.kind = 3;
            L.fp32 = 1;
            std::vector<unsigned char> ups, dns;
            std::vector<int> bs(1, 0);
            for (int b : probs) {
                const hps_op *op = ctx[b]->op;
                if (op->composed || !root_fused(op, true)) continue;
                ups.resize(ups.size() + ls);
                dns.resize(dns.size() + ls);
                int blocks = 0;
                size_t lds = 0;
                root_records(op, nullptr, ups.data() + ups.size() - ls, dns.data() + dns.size() - ls, &blocks, &lds,
                             ws[b], true, with_r3 ? r3_of(b) : nullptr);
                L.lds = std::max(L.lds, lds);
                bs.push_back(bs.back() + blocks);
            }
            L.cnt = (int)bs.size() - 1;
            if (L.cnt > 0) {
                L.a = T.put(ups.data(), ups.size());
                L.a2 = T.put(dns.data(), dns.size());
                L.base = T.put(bs.data(), sizeof(int) * bs.size());
                L.total = bs.back();
                P->seq.push_back(L);
            }
        }
        for (int l = 0; l < Lmax; ++l) {
            TRY(pairs(l, 1));
            TRY(level(l, false));
        }
        return HPS_OK;
    };
    // jumps_only: the leaf kernels evaluated the interior residual and the edge fluxes
    auto residual = [&](const std::vector<int> &probs, bool jumps_only) {
        GroupPlan::Launch L{};
        L.kind = 10;
        const size_t es = eval_record_size(), js = jump_record_size();
        std::vector<unsigned char> ev(es * probs.size()), jp(js * probs.size());
        std::vector<int> eb(probs.size() + 1, 0), jb(probs.size() + 1, 0);
        for (size_t i = 0; i < probs.size(); ++i) {
            const int b = probs[i];
            int leaves = 0, iface = 0;
            residual_records(ctx[b]->op, ctx[b]->stage_u, ctx[b]->rhs, r_of(b), r3_of(b), flux_of(b),
                             ev.data() + es * i, jp.data() + js * i, &leaves, &iface);
            if (!r3_of(b)) iface = 0;
            if (jumps_only) leaves = 0;
            eb[i + 1] = eb[i] + leaves;
            jb[i + 1] = jb[i] + iface;
        }
        L.a = T.put(ev.data(), ev.size());
        L.a2 = T.put(jp.data(), jp.size());
        L.base = T.put(eb.data(), sizeof(int) * eb.size());
        L.base2 = T.put(jb.data(), sizeof(int) * jb.size());
        L.cnt = (int)probs.size();
        L.total = eb.back();
        L.total2 = jb.back();
        P->seq.push_back(L);
    };
    // keep u^n for a redo, clear the correction norms
    {
        std::vector<MemOp> ops;
        for (int b = 0; b < n; ++b) {
            ops.push_back(MemOp{ctx[b]->u_save, u[b], ctx[b]->op->N});
            ops.push_back(MemOp{ctx[b]->ir_stat, nullptr, (int64_t)s * IR_MAXIT * 2});
        }
        std::vector<int64_t> ob(ops.size() + 1, 0);
        for (size_t i = 0; i < ops.size(); ++i) ob[i + 1] = ob[i] + ops[i].words;
        GroupPlan::Launch L{};
        L.kind = 9;
        L.a = T.put(ops.data(), sizeof(MemOp) * ops.size());
        L.base = T.put(ob.data(), sizeof(int64_t) * ob.size());
        L.cnt = (int)ops.size();
        L.words = ob.back();
        P->seq.push_back(L);
    }
    // per stage: the FP32 sweep; the leaf kernel that writes u, evaluates the refinement
    // residual and starts the first correction's FP32 solve; per correction the interface
    // jumps, the FP32 sweep, and the leaf kernel that adds the correction and either starts
    // the next correction (residual, FP32 solve) or, for the problem's last correction,
    // evaluates L u_i, F_i and opens the next stage; the norm folds.  The passes of the
    // single-problem replayed step, kernel for kernel.
    auto fold = [&](const std::vector<int> &probs, int k, int j) {
        std::vector<NormFold> folds;
        for (int b : probs)
            folds.push_back(NormFold{part_of(b),
                                     reinterpret_cast<unsigned long long *>(ctx[b]->ir_stat +
                                                                            ((int64_t)k * IR_MAXIT + j) * 2),
                                     (int)ctx[b]->op->nleaves});
        GroupPlan::Launch L{};
        L.kind = 11;
        L.a = T.put(folds.data(), sizeof(NormFold) * folds.size());
        L.cnt = (int)folds.size();
        P->seq.push_back(L);
    };
    auto stage_phase = [&](int b, int k, LeafPhase &ph) {
        step_phase(ctx[b], k, u[b], q_stages ? q_stages[b] : nullptr, q_space ? q_space[b] : nullptr, P->qt + 8 * b,
                   ph);
        if (k + 1 < s) ph.rhs_copy = ctx[b]->rhs;
    };
    for (int k = 0; k < s; ++k) {
        if (k == 0) {
            TRY(leaf(all, [&](int b, LeafPhase &ph) { stage_phase(b, 0, ph); }));
            continue;
        }
        TRY(sweep(all, false));
        TRY(leaf(all, [&](int b, LeafPhase &ph) {
            ph.down = LD_WRITE_U;
            ph.u_out = ctx[b]->stage_u;
            ph.res_rhs = ctx[b]->rhs;
            ph.up = LU_BODY;
        }));
        int kmax = 0;
        for (int b = 0; b < n; ++b) kmax = std::max(kmax, ctx[b]->ir_passes);
        for (int j = 0; j < kmax; ++j) {
            std::vector<int> probs, more, last;
            for (int b = 0; b < n; ++b)
                if (ctx[b]->ir_passes > j) {
                    probs.push_back(b);
                    (ctx[b]->ir_passes > j + 1 ? more : last).push_back(b);
                }
            residual(probs, true);
            TRY(sweep(probs, true));
            if (!more.empty())
                TRY(leaf(more, [&](int b, LeafPhase &ph) {
                    ph.down = LD_IR_ADD;
                    ph.u_out = ctx[b]->stage_u;
                    ph.norm_part = part_of(b);
                    ph.res_rhs = ctx[b]->rhs;
                    ph.up = LU_BODY;
                }));
            if (!last.empty())
                TRY(leaf(last, [&](int b, LeafPhase &ph) {
                    stage_phase(b, k, ph);
                    ph.down = LD_IR_ADD;
                    ph.ir_eval = true;
                    ph.u_out = ctx[b]->stage_u;
                    ph.norm_part = part_of(b);
                }));
            fold(probs, k, j);
        }
    }
    // boundary values (zero) and interface line solves of the update
    {
        const size_t zs = scatter_record_size(), lr = line_record_size();
        std::vector<unsigned char> zrec(zs * n), lrec(lr * n);
        std::vector<int> zb(n + 1, 0), lb(n + 1, 0);
        for (int b = 0; b < n; ++b) {
            int cnt = 0, sys = 0;
            scatter_record(ctx[b]->op, u[b], zrec.data() + zs * b, &cnt);
            line_record(ctx[b]->op, u[b], lrec.data() + lr * b, &sys, ws[b]);
            zb[b + 1] = zb[b] + cnt;
            lb[b + 1] = lb[b] + sys;
        }
        P->zb = GroupPlan::Launch{4, T.put(zrec.data(), zrec.size()), 0, T.put(zb.data(), sizeof(int) * (n + 1)),
                                  n, zb[n], 0, 0, 0};
        P->lines = GroupPlan::Launch{5, T.put(lrec.data(), lrec.size()), 0, T.put(lb.data(), sizeof(int) * (n + 1)),
                                     n, lb[n], 0, 0, 0};
    }
    P->host.swap(T.bytes);
    TRY(take_block(std::max<size_t>(P->host.size(), 256), st, &P->dmem, &P->dbytes));
    HPS_HIP(hipMemcpyAsync(P->dmem, P->host.data(), P->host.size(), hipMemcpyHostToDevice, st));
    P->done = new SharedEvent();
    P->done->refs = 1;
    HPS_HIP(hipEventCreateWithFlags(&P->done->e, hipEventDisableTiming));
    return HPS_OK;
}

int enqueue_plan(const GroupPlan *P, hipStream_t st) {
    unsigned char *d = P->dmem;
    auto basep = [&](const GroupPlan::Launch &L) { return reinterpret_cast<const int *>(d + L.base); };
    if (P->ir) {
        for (const GroupPlan::Launch &L : P->seq) {
            switch (L.kind) {
                case 0:
                    TRY(launch_leaf_group(d + L.a, basep(L), L.cnt, L.total, L.lds, L.down, L.up, st, true));
                    break;
                case 1:
                case 2:
                    TRY(launch_level_group(d + L.a, basep(L), L.cnt, L.total, L.lds, L.kind == 1, st, true));
                    break;
                case 3:
                    TRY(launch_root_group(d + L.a, d + L.a2, basep(L), L.cnt, L.total, L.lds, st, true));
                    break;
                case 9:
                    TRY(launch_memop_group(reinterpret_cast<const MemOp *>(d + L.a),
                                           reinterpret_cast<const int64_t *>(d + L.base), L.cnt, L.words, st));
                    break;
                case 10:
                    TRY(launch_residual_group(d + L.a, basep(L), d + L.a2, reinterpret_cast<const int *>(d + L.base2),
                                              L.cnt, L.total, L.total2, st));
                    break;
                case 11:
                    TRY(launch_norm_fold_group(reinterpret_cast<const NormFold *>(d + L.a), L.cnt, st));
                    break;
                case 6:
                case 7:
                case 8:
                    TRY(launch_pair_group(d + L.a, basep(L), L.cnt, L.total, L.lds, L.kind - 6, st, true));
                    break;
                default:
                    hps_set_error("internal: launch kind %d in a refined plan", L.kind);
                    return HPS_EINVAL;
            }
        }
        TRY(launch_zero_boundary_group(d + P->zb.a, basep(P->zb), P->zb.cnt, P->zb.total, st));
        TRY(launch_lines_group(d + P->lines.a, basep(P->lines), P->lines.cnt, P->lines.total, st));
        return HPS_OK;
    }
    auto run_sweep = [&]() -> int {
        for (const GroupPlan::Launch &L : P->sweep) {
            if (L.kind == 3) TRY(launch_root_group(d + L.a, d + L.a2, basep(L), L.cnt, L.total, L.lds, st));
            else if (L.kind == 12) TRY(launch_direct_group(d + L.a, basep(L), L.cnt, L.total, L.lds, st));
            else if (L.kind >= 6) TRY(launch_pair_group(d + L.a, basep(L), L.cnt, L.total, L.lds, L.kind - 6, st));
            else TRY(launch_level_group(d + L.a, basep(L), L.cnt, L.total, L.lds, L.kind == 1, st));
        }
        return HPS_OK;
    };
    for (int k = 0; k < P->s; ++k) {
        if (k > 0) TRY(run_sweep());
        const GroupPlan::Launch &L = P->leaf[k];
        TRY(launch_leaf_group(d + L.a, basep(L), L.cnt, L.total, L.lds, L.down, L.up, st));
    }
    TRY(launch_zero_boundary_group(d + P->zb.a, basep(P->zb), P->zb.cnt, P->zb.total, st));
    TRY(launch_lines_group(d + P->lines.a, basep(P->lines), P->lines.cnt, P->lines.total, st));
    return HPS_OK;
}

int grouped_step(ark_ctx *const *ctx, int n, double *const *u, const double *const *q_stages,
                 const double *const *q_space, const double *const *q_time, hipStream_t st, bool ir = false,
                 const int *ids = nullptr) {
    std::vector<uintptr_t> key;
    key.push_back(ir ? 1 : 0);
    for (int b = 0; b < n; ++b) {
        key.push_back((uintptr_t)ctx[b]);
        key.push_back((uintptr_t)ctx[b]->uid);
        key.push_back((uintptr_t)u[b]);
        key.push_back((uintptr_t)(q_stages ? q_stages[b] : nullptr));
        key.push_back((uintptr_t)(q_space ? q_space[b] : nullptr));
        if (ir) key.push_back((uintptr_t)ctx[b]->ir_passes);
    }
    std::lock_guard<std::mutex> g(g_plans_mu);
    reap_retired();
    GroupPlan *P = nullptr;
    for (GroupPlan *p : g_plans)
        if (p->key == key) P = p;
    if (!P) {
        if (g_plans.size() >= kMaxPlans) {
            auto lru = std::min_element(g_plans.begin(), g_plans.end(),
                                        [](GroupPlan *a, GroupPlan *b) { return a->last_use < b->last_use; });
            retire_plan(*lru);
            g_plans.erase(lru);
        }
        P = new GroupPlan();
        P->key = key;
        if (int rc = ir ? build_plan_ir(P, ctx, n, u, q_stages, q_space, st)
                        : build_plan(P, ctx, n, u, q_stages, q_space, st)) {
            retire_plan(P);
            return rc;
        }
        g_plans.push_back(P);
    }
    P->last_use = ++g_plan_clock;
    // separable sources: this step's time factors, copied before the (replayed) step
    if (q_space && q_time) {
        std::vector<double> qt(8 * (size_t)n, 0.0);
        bool any = false;
        for (int b = 0; b < n; ++b)
            if (q_space[b] && q_time[b]) {
                any = true;
                for (int i = 0; i < P->s; ++i) qt[8 * b + i] = q_time[b][i];
            }
        if (any) HPS_HIP(hipMemcpyAsync(P->qt, qt.data(), sizeof(double) * qt.size(), hipMemcpyHostToDevice, st));
    }
    const char *env = getenv("HPS_GRAPHS");
    const bool graphs = !(env && env[0] == '0') && P->uses > 0;   // a set's first step runs eagerly
    P->uses++;
    if (!graphs) {
        TRY(enqueue_plan(P, st));
    } else {
        if (!P->gexec) {
            if (!P->cap) HPS_HIP(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
            HPS_HIP(hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed));
            const int rc = enqueue_plan(P, P->cap);
            hipGraph_t gr = nullptr;
            const hipError_t e = hipStreamEndCapture(P->cap, &gr);
            if (rc) {
                if (gr) (void)hipGraphDestroy(gr);
                return rc;
            }
            HPS_HIP(e);
            P->graph = gr;
            HPS_HIP(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
        }
        HPS_HIP(hipGraphLaunch(P->gexec, st));
    }
    HPS_HIP(hipEventRecord(P->done->e, st));
    if (!ir) return HPS_OK;
    // every problem's correction norms, one wait for all; a problem whose refinement missed
    // the tolerance is redone alone (from its saved u^n, host-checked)
    const size_t per = (size_t)P->s * IR_MAXIT * 2;
    std::vector<unsigned long long> stats(per * n);
    for (int b = 0; b < n; ++b)
        HPS_HIP(hipMemcpyAsync(stats.data() + per * b, ctx[b]->ir_stat, per * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, st));
    HPS_HIP(hipStreamSynchronize(st));
    int rc = HPS_OK;
    for (int b = 0; b < n; ++b) {
        const int r = ir_step_finish(ctx[b], u[b], q_stages ? q_stages[b] : nullptr, q_space ? q_space[b] : nullptr,
                                     q_time ? q_time[b] : nullptr, nullptr, st, stats.data() + per * b);
        if (r && !rc) rc = tag_problem(r, ids ? ids[b] : b);   // the caller's problem index
    }
    return rc;
}

}  // namespace

extern "C" int hps_batch_streams(void) { return kStreams; }

extern "C" int hps_solve_batched(hps_op *const *ops, int nprob, const double *const *body,
                                 const double *const *dirichlet, const double *const *jump,
                                 double *const *u, void *stream, hps_info *info) {
    CHECK_ARG(nprob >= 0 && nprob <= HPS_BATCH_MAX, "nprob must be in [0, HPS_BATCH_MAX]");
    if (nprob == 0) return HPS_OK;
    CHECK_ARG(ops != nullptr && body != nullptr && u != nullptr, "ops, body and u are required");
    std::vector<const hps_op *> v(nprob);
    for (int b = 0; b < nprob; ++b) {
        if (!ops[b] || !body[b] || !u[b]) {
            hps_set_error("problem %d: op, body and u are required", b);
            return HPS_EINVAL;
        }
        v[b] = ops[b];
    }
    hipStream_t caller = (hipStream_t)stream;
    int rc = run_batched(v, caller, [&](int b, hipStream_t st) {
        return hps_solve(ops[b], 1, body[b], dirichlet ? dirichlet[b] : nullptr,
                         jump ? jump[b] : nullptr, u[b], st, info ? &info[b] : nullptr);
    });
    if (rc == HPS_OK && info) HPS_HIP(hipStreamSynchronize(caller));
    return rc;
}

extern "C" int ark_step_batched(ark_ctx *const *ctx, int nprob, const double *t, double *const *u,
                                const double *const *q_stages, const double *const *q_space,
                                const double *const *q_time, const double *const *f_stages,
                                void *stream) {
    CHECK_ARG(nprob >= 0 && nprob <= HPS_BATCH_MAX, "nprob must be in [0, HPS_BATCH_MAX]");
    if (nprob == 0) return HPS_OK;
    CHECK_ARG(ctx != nullptr && t != nullptr && u != nullptr, "ctx, t and u are required");
    std::vector<const hps_op *> v(nprob);
    for (int b = 0; b < nprob; ++b) {
        if (!ctx[b] || !u[b]) {
            hps_set_error("problem %d: ctx and u are required", b);
            return HPS_EINVAL;
        }
        v[b] = ctx[b]->op;
    }
    for (int b = 0; b < nprob; ++b) {
        CHECK_ARG(std::isfinite(t[b]), "problem %d: t must be finite", b);
        TRY(check_device_ptr(u[b], "u"));
        if (q_stages) TRY(check_device_ptr(q_stages[b], "q_stages"));
        if (q_space) TRY(check_device_ptr(q_space[b], "q_space"));
        if (q_space && q_space[b]) CHECK_ARG(q_time && q_time[b], "problem %d: q_space needs q_time", b);
        CHECK_ARG(!(q_stages && q_stages[b] && q_space && q_space[b]), "problem %d: q_stages or q_space, not both", b);
    }
    // problems that can share launches, by kind (FP64 / refined FP32) and stage count; each
    // such set of two or more runs as one grouped step, the others one by one on the pool
    std::map<std::pair<int, int>, std::vector<int>> sets;
    std::vector<int> rest;
    for (int b = 0; b < nprob; ++b) {
        ark_ctx *const one[1] = {ctx[b]};
        const double *const fb[1] = {f_stages ? f_stages[b] : nullptr};
        if (groupable(one, 1, nullptr, fb)) sets[{0, ctx[b]->s}].push_back(b);
        else if (groupable_ir(one, 1, fb)) sets[{1, ctx[b]->s}].push_back(b);
        else rest.push_back(b);
    }
    const hipStream_t st = (hipStream_t)stream;
    for (auto &kv : sets) {
        const std::vector<int> &m = kv.second;
        if (m.size() < 2) {
            rest.insert(rest.end(), m.begin(), m.end());
            continue;
        }
        std::vector<ark_ctx *> c(m.size());
        std::vector<double *> uu(m.size());
        std::vector<const double *> qs(m.size()), qp(m.size()), qt(m.size());
        for (size_t i = 0; i < m.size(); ++i) {
            c[i] = ctx[m[i]];
            uu[i] = u[m[i]];
            qs[i] = q_stages ? q_stages[m[i]] : nullptr;
            qp[i] = q_space ? q_space[m[i]] : nullptr;
            qt[i] = q_time ? q_time[m[i]] : nullptr;
        }
        const int rc = grouped_step(c.data(), (int)m.size(), uu.data(), qs.data(), qp.data(), qt.data(), st,
                                    kv.first.first == 1, m.data());
        if (rc) return rc;
    }
    if (rest.empty()) return HPS_OK;
    std::sort(rest.begin(), rest.end());
    std::vector<const hps_op *> rv(rest.size());
    for (size_t i = 0; i < rest.size(); ++i) rv[i] = v[rest[i]];
    return run_batched(
        rv, st,
        [&](int i, hipStream_t s2) {
            const int b = rest[i];
            return ark_step(ctx[b], t[b], u[b], q_stages ? q_stages[b] : nullptr, q_space ? q_space[b] : nullptr,
                            q_time ? q_time[b] : nullptr, f_stages ? f_stages[b] : nullptr, s2);
        },
        &rest);
}
