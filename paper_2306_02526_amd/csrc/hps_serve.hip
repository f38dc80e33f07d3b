// Time-stepping server: an operator cache keyed by (grid, coefficient key, gamma*dt,
// flags), first-come first-served admission under a device-memory budget, and continuous
// batching (every running job advances one step per ark_step_batched call).  Runs on a
// host thread of its own; the GPU work is exactly what hps_build and ark_step enqueue.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "hps_batch.h"
#include "hps_internal.h"
#include "hps_serve.h"

using namespace hps;

namespace {

using Clock = std::chrono::steady_clock;
using Key = std::tuple<double, double, double, double, int, int, int, uint64_t, uint64_t, int>;

constexpr size_t kMaxSpare = 4;   // contexts of finished jobs kept per operator

struct CacheEntry {
    hps_op *op = nullptr;
    int64_t bytes = 0;              // the operator's device bytes
    int64_t ctx_bytes = 0;          // its contexts' bytes: running jobs' and kept ones
    int refs = 0;
    uint64_t last_use = 0;
    std::vector<ark_ctx *> spare;   // stepping contexts of finished jobs, reused by later ones
};

struct Job {
    int64_t id = 0;
    srv_job spec{};
    std::vector<double> A, b, c, Ah, bh;
    Key key{};
    double gamma_dt = 0;
    hipEvent_t ready = nullptr;   // caller's stream at submission
    ark_ctx *ctx = nullptr;
    hps_op *op = nullptr;
    bool waited = false;
    int enqueued = 0;             // steps enqueued (st.steps_done counts completed ones)
    srv_status st{};
};

// A context can serve another job of the same operator if the step it takes is the same.
bool same_step(const ark_ctx *c, const Job *j) {
    const int s = j->spec.tab.s;
    return c->s == s && c->dt == j->spec.dt && c->A == j->A && c->b == j->b && c->c == j->c &&
           c->Ah == j->Ah && c->bh == j->bh && c->g.kind == j->spec.g.kind && c->g.g0 == j->spec.g.g0 &&
           c->g.g1 == j->spec.g.g1 && c->g.g2 == j->spec.g.g2 && c->g.g3 == j->spec.g.g3;
}

// Device bytes an operator of this grid will hold: its packed panels plus the solve
// workspace (about ten doubles per node).
int64_t operator_footprint(const hps_grid &g, int flags) {
    const int64_t N = hps_num_nodes(&g, nullptr, nullptr, nullptr);
    return plan_operator_bytes(g, flags) + 80 * N;
}

}  // namespace

struct srv_server {
    int device = 0;
    srv_config cfg{};
    Clock::time_point t0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable wake, finished;
    bool stopping = false;
    int64_t next_id = 0;
    std::deque<Job *> queue;                 // submitted, not yet admitted
    std::map<int64_t, Job *> jobs;           // every job not yet released
    std::vector<Job *> active;               // worker thread only
    std::map<Key, CacheEntry> cache;         // worker thread only (stats under mu)
    uint64_t use_clock = 0;
    srv_stats stats{};
    hipStream_t stream = nullptr;
    // iterations enqueued but not yet known complete (at most two)
    struct Inflight {
        hipEvent_t ev = nullptr;
        std::vector<Job *> stepped, last;   // jobs stepped; jobs whose last step this is
    };
    std::deque<Inflight> inflight;
    std::vector<hipEvent_t> ev_pool;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    int admit(Job *j);
    void finish(Job *j, int state, int err);
    void release_op(Job *j);
    int retire_oldest();
    void evict_entry(std::map<Key, CacheEntry>::iterator it);
    int64_t held() const;
    void update_held_stats();
};

void srv_server::evict_entry(std::map<Key, CacheEntry>::iterator it) {
    for (ark_ctx *c : it->second.spare) ark_free(c);
    hps_free(it->second.op);
    cache.erase(it);
}

// device bytes charged to the budget: operators and contexts
int64_t srv_server::held() const {
    int64_t b = 0;
    for (auto &e : cache) b += e.second.bytes + e.second.ctx_bytes;
    return b;
}

void srv_server::update_held_stats() {
    int64_t ob = 0, cb = 0;
    for (auto &e : cache) {
        ob += e.second.bytes;
        cb += e.second.ctx_bytes;
    }
    std::lock_guard<std::mutex> g(mu);
    stats.cached_ops = (int64_t)cache.size();
    stats.cached_bytes = ob;
    stats.context_bytes = cb;
}

void srv_server::release_op(Job *j) {
    auto it = j->op ? cache.find(j->key) : cache.end();
    if (j->ctx) {
        // keep the context for the next job of this operator (freeing device memory would
        // wait for the whole device), a few per operator; it stays charged to the budget
        if (it != cache.end() && it->second.spare.size() < kMaxSpare) {
            it->second.spare.push_back(j->ctx);
        } else {
            if (it != cache.end()) it->second.ctx_bytes -= ark_ctx_footprint(j->op, j->ctx->s);
            ark_free(j->ctx);
        }
    }
    j->ctx = nullptr;
    if (it != cache.end()) {
        it->second.refs--;
        it->second.last_use = ++use_clock;
    }
    j->op = nullptr;
    if (j->ready) (void)hipEventDestroy(j->ready);
    j->ready = nullptr;
    update_held_stats();
}

void srv_server::finish(Job *j, int state, int err) {
    release_op(j);
    std::lock_guard<std::mutex> g(mu);
    j->st.state = state;
    j->st.error = err;
    j->st.finish_s = now();
    if (state == SRV_DONE) stats.completed++;
    else stats.failed++;
    finished.notify_all();
}

// Acquire the job's operator (cache hit, or build after evicting unreferenced operators,
// least recently used first) and its stepping context.  Returns 1 if the job must wait
// for referenced operators to be released, 0 on success, < 0 on a failure of the job.
int srv_server::admit(Job *j) {
    auto it = cache.find(j->key);
    bool hit = it != cache.end();
    // the bytes this job adds: its operator when not cached, its context unless a kept one
    // of the same step can be reused
    bool reuse = false;
    if (hit)
        for (ark_ctx *c : it->second.spare) reuse = reuse || same_step(c, j);
    const int64_t op_need = hit ? 0 : operator_footprint(j->spec.grid, j->spec.flags | HPS_WIDE_TILES);
    int64_t ctx_need = 0;
    if (!reuse) {
        if (hit) {
            ctx_need = ark_ctx_footprint(it->second.op, j->spec.tab.s);
        } else {
            // the context of an operator not built yet: sized from the grid (its workspace
            // is a small multiple of N doubles, charged generously)
            int64_t n_int = 0;
            const int64_t N = hps_num_nodes(&j->spec.grid, &n_int, nullptr, nullptr);
            ctx_need = 8 * (2LL * j->spec.tab.s * n_int + j->spec.tab.s + 3 * N + 20 * N);
        }
    }
    const int64_t need = op_need + ctx_need;
    if (need > cfg.cache_bytes) {
        hps_set_error("operator and stepping context of %lld bytes exceed the cache budget", (long long)need);
        return HPS_ENOMEM;
    }
    int64_t h = held();
    // make room: kept contexts first (least recently used operators first), then
    // unreferenced operators
    while (h + need > cfg.cache_bytes) {
        auto donor = cache.end();
        for (auto e = cache.begin(); e != cache.end(); ++e)
            if (!e->second.spare.empty() && !(hit && e == it && reuse) &&
                (donor == cache.end() || e->second.last_use < donor->second.last_use))
                donor = e;
        if (donor != cache.end()) {
            ark_ctx *c = donor->second.spare.back();
            donor->second.spare.pop_back();
            const int64_t cb = ark_ctx_footprint(donor->second.op, c->s);
            donor->second.ctx_bytes -= cb;
            h -= cb;
            ark_free(c);
            continue;
        }
        auto victim = cache.end();
        for (auto e = cache.begin(); e != cache.end(); ++e)
            if (e->second.refs == 0 && !(hit && e == it) &&
                (victim == cache.end() || e->second.last_use < victim->second.last_use))
                victim = e;
        if (victim == cache.end()) {
            std::lock_guard<std::mutex> g(mu);
            stats.waits++;
            return 1;
        }
        h -= victim->second.bytes + victim->second.ctx_bytes;
        evict_entry(victim);
        std::lock_guard<std::mutex> g(mu);
        stats.evictions++;
    }
    if (!hit) {
        // the coefficient arrays were prepared on the caller's stream
        if (hipStreamWaitEvent(stream, j->ready, 0) != hipSuccess) {
            hps_set_error("hipStreamWaitEvent failed");
            return HPS_EDEVICE;
        }
        j->waited = true;
        hps_op *op = nullptr;
        // served jobs are stepped many at a time: level operators in few large tiles
        if (int rc = hps_build(&j->spec.grid, &j->spec.coeffs, j->gamma_dt, j->spec.flags | HPS_WIDE_TILES,
                               stream, &op))
            return rc;
        CacheEntry e;
        e.op = op;
        int64_t ob = 0;
        e.bytes = hps_op_bytes(op, &ob);
        it = cache.emplace(j->key, e).first;
        std::lock_guard<std::mutex> g(mu);
        stats.builds++;
    } else {
        std::lock_guard<std::mutex> g(mu);
        stats.cache_hits++;
    }
    it->second.refs++;
    it->second.last_use = ++use_clock;
    j->op = it->second.op;
    auto &sp = it->second.spare;
    for (size_t k = 0; k < sp.size() && !j->ctx; ++k)
        if (same_step(sp[k], j)) {
            j->ctx = sp[k];
            sp.erase(sp.begin() + (long)k);
        }
    if (!j->ctx) {
        ark_tableau tab{j->spec.tab.s, j->A.data(), j->b.data(), j->c.data(), j->Ah.data(), j->bh.data()};
        if (int rc = ark_create(j->op, &tab, j->spec.dt, &j->spec.g, &j->ctx)) {
            it->second.refs--;
            j->op = nullptr;
            return rc;
        }
        it->second.ctx_bytes += ark_ctx_footprint(j->op, j->spec.tab.s);
    }
    update_held_stats();
    std::lock_guard<std::mutex> g(mu);
    j->st.cache_hit = hit ? 1 : 0;
    j->st.state = SRV_ACTIVE;
    j->st.start_s = now();
    return 0;
}

// Wait for the oldest in-flight iteration; count its steps and finish the jobs whose
// last step it held.  Returns the iteration's error (HPS_OK or HPS_EDEVICE).
int srv_server::retire_oldest() {
    Inflight f = inflight.front();
    inflight.pop_front();
    const int rc = hipEventSynchronize(f.ev) == hipSuccess ? HPS_OK : HPS_EDEVICE;
    ev_pool.push_back(f.ev);
    {
        std::lock_guard<std::mutex> g(mu);
        for (Job *j : f.stepped) j->st.steps_done++;
        stats.job_steps += (int64_t)f.stepped.size();
    }
    for (Job *j : f.last) finish(j, rc == HPS_OK ? SRV_DONE : SRV_FAILED, rc);
    return rc;
}

void srv_server::run() {
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Job *> incoming;
        {
            std::unique_lock<std::mutex> lk(mu);
            wake.wait(lk, [&] { return stopping || !queue.empty() || !active.empty() || !inflight.empty(); });
            if (stopping && queue.empty() && active.empty() && inflight.empty()) break;
            // first come, first served: take jobs from the head while slots are free
            while (!queue.empty() && (int)(active.size() + incoming.size()) < cfg.max_active) {
                incoming.push_back(queue.front());
                queue.pop_front();
            }
        }
        for (size_t k = 0; k < incoming.size(); ++k) {
            Job *j = incoming[k];
            const int rc = admit(j);
            if (rc == 1) {
                // wait for running jobs to release operators; keep the arrival order
                std::lock_guard<std::mutex> g(mu);
                for (size_t r = incoming.size(); r-- > k;) queue.push_front(incoming[r]);
                break;
            }
            if (rc < 0) finish(j, SRV_FAILED, rc);
            else active.push_back(j);
        }
        if (!active.empty()) {
            // one step of every running job, as one batched call; the next iteration is
            // enqueued before this one is waited for, so the GPU does not idle in between
            const int n = (int)active.size();
            std::vector<ark_ctx *> ctxs(n);
            std::vector<double> ts(n);
            std::vector<double *> us(n);
            std::vector<const double *> qsp(n, nullptr), qtp(n, nullptr);
            std::vector<std::vector<double>> qt(n);
            bool any_q = false;
            int rc = HPS_OK;
            for (int b = 0; b < n; ++b) {
                Job *j = active[b];
                if (!j->waited) {
                    if (hipStreamWaitEvent(stream, j->ready, 0) != hipSuccess) rc = HPS_EDEVICE;
                    j->waited = true;
                }
                ctxs[b] = j->ctx;
                ts[b] = j->spec.t0 + j->enqueued * j->spec.dt;
                us[b] = j->spec.u;
                if (j->spec.q_space) {
                    any_q = true;
                    qsp[b] = j->spec.q_space;
                    qt[b].resize(j->spec.tab.s);
                    for (int i = 0; i < j->spec.tab.s; ++i)
                        qt[b][i] = j->spec.q_amp * std::exp(j->spec.q_rate * (ts[b] + j->c[i] * j->spec.dt));
                    qtp[b] = qt[b].data();
                }
            }
            if (rc == HPS_OK)
                rc = ark_step_batched(ctxs.data(), n, ts.data(), us.data(), nullptr, any_q ? qsp.data() : nullptr,
                                      any_q ? qtp.data() : nullptr, nullptr, stream);
            Inflight f;
            if (ev_pool.empty()) {
                hipEvent_t e = nullptr;
                if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = HPS_EDEVICE;
                ev_pool.push_back(e);
            }
            f.ev = ev_pool.back();
            ev_pool.pop_back();
            if (rc == HPS_OK && hipEventRecord(f.ev, stream) != hipSuccess) rc = HPS_EDEVICE;
            if (rc != HPS_OK) {
                ev_pool.push_back(f.ev);
                while (!inflight.empty()) retire_oldest();
                for (Job *j : active) finish(j, SRV_FAILED, rc);
                active.clear();
            } else {
                std::vector<Job *> still;
                for (Job *j : active) {
                    f.stepped.push_back(j);
                    if (++j->enqueued >= j->spec.steps) f.last.push_back(j);
                    else still.push_back(j);
                }
                active.swap(still);
                inflight.push_back(f);
                std::lock_guard<std::mutex> g(mu);
                stats.iterations++;
            }
        }
        // keep one iteration in flight while more work is queued or running
        const size_t keep = active.empty() ? 0 : 1;
        while (inflight.size() > keep) retire_oldest();
        if (active.empty() && inflight.empty()) {
            std::unique_lock<std::mutex> lk(mu);
            if (!stopping && !queue.empty()) wake.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

extern "C" int srv_create(const srv_config *cfg, srv_server **out) {
    CHECK_ARG(out != nullptr, "out is NULL");
    srv_config c{};
    if (cfg) c = *cfg;
    CHECK_ARG(c.cache_bytes >= 0, "cache_bytes must be >= 0");
    CHECK_ARG(c.max_active >= 0 && c.max_active <= 4096, "max_active must be in [0, 4096]");
    CHECK_ARG(c.max_queued >= 0, "max_queued must be >= 0");
    if (c.max_active == 0) c.max_active = 64;
    int dev = 0;
    HPS_HIP(hipGetDevice(&dev));
    if (c.cache_bytes == 0) {
        size_t fr = 0, tot = 0;
        HPS_HIP(hipMemGetInfo(&fr, &tot));
        c.cache_bytes = (int64_t)(fr / 4 * 3);
    }
    srv_server *s = new srv_server();
    s->device = dev;
    s->cfg = c;
    s->t0 = Clock::now();
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        hps_set_error("could not create the server's stream");
        return HPS_EDEVICE;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return HPS_OK;
}

extern "C" int srv_submit(srv_server *srv, const srv_job *job, void *stream, int64_t *id) {
    CHECK_ARG(srv != nullptr && job != nullptr && id != nullptr, "srv, job and id are required");
    int64_t n_int = 0, n_iface = 0, n_bdry = 0;
    const int64_t N = hps_num_nodes(&job->grid, &n_int, &n_iface, &n_bdry);
    if (N < 0) return (int)N;
    const ark_tableau &t = job->tab;
    CHECK_ARG(t.s >= 2 && t.s <= 8 && t.A && t.b && t.c && t.Ahat && t.bhat, "tableau needs 2 <= s <= 8 and all arrays");
    CHECK_ARG(job->dt > 0 && std::isfinite(job->dt), "dt must be positive");
    CHECK_ARG(job->steps >= 1, "steps must be >= 1");
    CHECK_ARG((job->flags & ~(HPS_FP32_IR | HPS_UNIFORM_COEFFS)) == 0,
              "flags must be HPS_FP64 or HPS_FP32_IR, optionally with HPS_UNIFORM_COEFFS");
    CHECK_ARG(job->g.kind == 0 || job->g.kind == 1, "ark_g.kind must be 0 or 1");
    CHECK_ARG(job->u != nullptr, "u is required");
    CHECK_ARG(std::isfinite(job->t0) && std::isfinite(job->q_amp) && std::isfinite(job->q_rate),
              "t0, q_amp and q_rate must be finite");
    TRY(check_device_ptr(job->u, "u"));
    TRY(check_device_ptr(job->q_space, "q_space"));
    const double *co[5] = {job->coeffs.cxx, job->coeffs.cyy, job->coeffs.cx, job->coeffs.cy, job->coeffs.c0};
    for (const double *p : co) TRY(check_device_ptr(p, "coefficient"));
    const double gdt = t.A[1 * t.s + 1] * job->dt;
    CHECK_ARG(gdt > 0, "the tableau's gamma must be positive");
    Job *j = new Job();
    j->spec = *job;
    const int s = t.s;
    j->A.assign(t.A, t.A + s * s);
    j->b.assign(t.b, t.b + s);
    j->c.assign(t.c, t.c + s);
    j->Ah.assign(t.Ahat, t.Ahat + s * s);
    j->bh.assign(t.bhat, t.bhat + s);
    j->spec.tab = ark_tableau{s, nullptr, nullptr, nullptr, nullptr, nullptr};
    j->gamma_dt = gdt;
    uint64_t gbits = 0;
    std::memcpy(&gbits, &gdt, sizeof(gbits));
    const hps_grid &g = job->grid;
    j->key = Key(g.x0, g.x1, g.y0, g.y1, g.n1, g.n2, g.p, job->coef_key, gbits, job->flags);
    if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(j->ready, (hipStream_t)stream) != hipSuccess) {
        if (j->ready) (void)hipEventDestroy(j->ready);
        delete j;
        hps_set_error("could not record the job's ready event");
        return HPS_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) {
        (void)hipEventDestroy(j->ready);
        delete j;
        hps_set_error("server is shutting down");
        return HPS_EINVAL;
    }
    if (srv->cfg.max_queued > 0 && (int64_t)srv->queue.size() >= srv->cfg.max_queued) {
        (void)hipEventDestroy(j->ready);
        delete j;
        hps_set_error("%d jobs are already waiting for admission", srv->cfg.max_queued);
        return HPS_EBUSY;
    }
    j->id = srv->next_id++;
    j->st.state = SRV_QUEUED;
    j->st.submit_s = srv->now();
    srv->jobs[j->id] = j;
    srv->queue.push_back(j);
    srv->stats.submitted++;
    *id = j->id;
    srv->wake.notify_one();
    return HPS_OK;
}

extern "C" int srv_poll(srv_server *srv, int64_t id, srv_status *status) {
    CHECK_ARG(srv != nullptr && status != nullptr, "srv and status are required");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(id);
    CHECK_ARG(it != srv->jobs.end(), "unknown job id %lld", (long long)id);
    *status = it->second->st;
    return HPS_OK;
}

extern "C" int srv_wait(srv_server *srv, int64_t id, srv_status *status) {
    CHECK_ARG(srv != nullptr, "srv is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(id);
    CHECK_ARG(it != srv->jobs.end(), "unknown job id %lld", (long long)id);
    Job *j = it->second;
    srv->finished.wait(lk, [&] { return j->st.state == SRV_DONE || j->st.state == SRV_FAILED; });
    if (status) *status = j->st;
    return HPS_OK;
}

extern "C" int srv_release(srv_server *srv, int64_t id) {
    CHECK_ARG(srv != nullptr, "srv is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(id);
    CHECK_ARG(it != srv->jobs.end(), "unknown job id %lld", (long long)id);
    CHECK_ARG(it->second->st.state == SRV_DONE || it->second->st.state == SRV_FAILED,
              "job %lld has not finished", (long long)id);
    delete it->second;
    srv->jobs.erase(it);
    return HPS_OK;
}

extern "C" int srv_get_stats(srv_server *srv, srv_stats *stats) {
    CHECK_ARG(srv != nullptr && stats != nullptr, "srv and stats are required");
    std::lock_guard<std::mutex> lk(srv->mu);
    *stats = srv->stats;
    return HPS_OK;
}

extern "C" void srv_destroy(srv_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        srv->wake.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    while (!srv->cache.empty()) srv->evict_entry(srv->cache.begin());
    for (auto &kv : srv->jobs) delete kv.second;
    for (hipEvent_t e : srv->ev_pool) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(srv->stream);
    delete srv;
}
