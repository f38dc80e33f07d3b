// Batched entry points: many independent problems per call, spread over a pool of
// library-owned HIP streams so that small problems overlap on the GPU.  Every problem
// runs through the same entry points as a single call (hps_solve, ark_step); this file
// only forks, assigns and joins streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/hps_batch.h"
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
int run_batched(const std::vector<const hps_op *> &ops, hipStream_t caller, Fn fn) {
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
        if (rc != HPS_OK) rc = tag_problem(rc, b);
    }
    // join even after an error, so the caller's stream still orders after what ran
    for (int k = 0; k < kStreams; ++k) {
        if (!used[k]) continue;
        HPS_HIP(hipEventRecord(pool->done[k], pool->s[k]));
        HPS_HIP(hipStreamWaitEvent(caller, pool->done[k], 0));
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
    return run_batched(v, (hipStream_t)stream, [&](int b, hipStream_t st) {
        return ark_step(ctx[b], t[b], u[b], q_stages ? q_stages[b] : nullptr,
                        q_space ? q_space[b] : nullptr, q_time ? q_time[b] : nullptr,
                        f_stages ? f_stages[b] : nullptr, st);
    });
}
