// serve.cpp - continuous-batching request loop over the batched solve.
//
// A scheduler thread owns the device work.  Each turn it
//   1. retires launched batches whose completion event has fired (their
//      workspaces go back to a pool, their slots free up, latency is the
//      host time from submit to the observed completion) and takes over the
//      plans whose spectrum a precompute thread has finished;
//   2. admits queued requests in arrival order while a slot is free and the
//      request's footprint fits the HBM budget: a workspace for (n, tier)
//      (reused from the pool when one is free) and the multiplier octant
//      (8 (n+1)^2 round_up(n+1,16) bytes).  On a spectrum-cache miss the
//      octant's bytes are reserved and the precompute (Algorithm 1) is handed
//      to the precompute thread, which runs it on a stream of its own; the
//      request stays queued, and later requests whose spectra are cached are
//      admitted past it meanwhile.  Idle cached spectra and pooled workspaces
//      are evicted, least recently used first, to make room; the queue head
//      waits when nothing more can be freed;
//   3. launches the admitted requests of one tier and size class (n <= 128 or
//      larger) as one batch on a stream of that class (two streams per
//      class, the one with fewer batches in flight) and records a completion
//      event, so requests that arrive while others run are admitted and
//      overlap on the device, and a small request never waits in stream
//      order behind a large one.
// Every solve runs the same kernels on its own workspace, so a result is
// bitwise the same alone and in any mix.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <tuple>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <thread>
#include <unordered_map>

#include "host_common.hpp"

namespace psp {

using Clock = std::chrono::steady_clock;
hipError_t launch_batch(int count, const SolveArgs *args, hipStream_t st);

// batch kinds per scheduler turn: tier (FP64, FP32) x size class (n <= kSmallN
// or larger)
constexpr int kBatchKinds = 4;
constexpr int kSmallN = 128;

struct ServeReq {
    int n = 0;
    double h = 0;
    int R = 0;
    psp_dtype tier = PSP_F64;
    const void *rho = nullptr;
    void *u = nullptr;
    Clock::time_point t_submit;
    bool done = false;
    bool missed = false;            // its spectrum was not cached on arrival
    psp_status result = PSP_OK;
    double latency_ms = 0;
};

using SpecKey3 = std::tuple<int, double, int>;

struct CachedSpec {                 // plans of both tiers for one (n, h, R)
    psp_plan *plan[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};   // a precompute of that tier is running
    size_t bytes = 0;               // the octant's bytes, accounted once per key
    int users = 0;
    Clock::time_point last_use;
};

// a precompute handed to the precompute thread, and its outcome
struct PreJob {
    SpecKey3 key;
    int tier = 0;
};
struct PreDone {
    SpecKey3 key;
    int tier = 0;
    psp_plan *plan = nullptr;
    psp_status st = PSP_OK;
    std::string detail;
};

// streams: kClassStreams for n <= kSmallN, as many for larger n
constexpr int kClassStreams = 2;

struct PooledWs {
    Workspace w;
    int n;
    bool f32;
};

struct Batch {
    hipEvent_t ev = nullptr;
    int stream = 0;                 // index into the server's stream pool
    std::vector<uint64_t> ids;
    std::vector<PooledWs> ws;
    std::vector<std::tuple<int, double, int>> keys;
};

}  // namespace psp

using namespace psp;

struct psp_server {
    size_t budget = 0;
    int max_slots = 1;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, ServeReq> reqs;
    std::deque<uint64_t> finished;          // completed tickets, oldest first
    uint64_t next_id = 1;
    size_t pending_total = 0;
    bool stop = false;
    // precompute thread: jobs in, finished plans out (under pre_mu)
    std::mutex pre_mu;
    std::condition_variable pre_cv;
    std::deque<PreJob> pre_jobs;
    std::vector<PreDone> pre_done;
    bool pre_stop = false;
    hipStream_t pre_stream = nullptr;
    std::thread pre_thread;
    // scheduler-thread state
    std::map<SpecKey3, CachedSpec> specs;
    std::vector<PooledWs> pool;
    std::list<Batch> inflight;
    std::vector<hipStream_t> streams;
    int slots_used = 0;
    std::atomic<size_t> bytes_in_use{0}, bytes_peak{0};
    std::atomic<uint64_t> completed{0}, hits{0}, misses{0};
    std::thread sched;
};

namespace psp {

static void account(psp_server *sv, long delta) {
    size_t now = sv->bytes_in_use.fetch_add((size_t)delta) + (size_t)delta;
    size_t pk = sv->bytes_peak.load();
    while (now > pk && !sv->bytes_peak.compare_exchange_weak(pk, now)) {
    }
}

// requests run in grouped batch launches, whose workspaces hold all k3 tiles
static size_t ws_bytes(int n, bool f32) { return workspace_bytes(n, f32, 0); }

static void free_ws(psp_server *sv, PooledWs &p) {
    const size_t b = p.w.bytes;
    free_workspace(&p.w);
    account(sv, -(long)b);
}

// free idle memory (pooled workspaces first, then LRU idle spectra) until
// `need` more bytes fit the budget; returns whether they fit
static bool make_room(psp_server *sv, size_t need, const std::tuple<int, double, int> *keep) {
    while (sv->bytes_in_use.load() + need > sv->budget) {
        if (!sv->pool.empty()) {
            free_ws(sv, sv->pool.back());
            sv->pool.pop_back();
            continue;
        }
        auto victim = sv->specs.end();
        for (auto it = sv->specs.begin(); it != sv->specs.end(); ++it) {
            if (it->second.users > 0 || it->second.pending[0] || it->second.pending[1] || (keep && it->first == *keep))
                continue;
            if (victim == sv->specs.end() || it->second.last_use < victim->second.last_use) victim = it;
        }
        if (victim == sv->specs.end()) return false;
        for (int t = 0; t < 2; ++t) psp_plan_destroy(victim->second.plan[t]);
        account(sv, -(long)victim->second.bytes);
        sv->specs.erase(victim);
    }
    return true;
}

// The precompute thread: creates the plan of a job and runs its precompute
// (Algorithm 1: 1D tables and the spectrum contraction, synchronous on the
// thread's own stream), then hands the plan to the scheduler.
static void precompute_worker(psp_server *sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        PreJob job;
        {
            std::unique_lock<std::mutex> lk(sv->pre_mu);
            sv->pre_cv.wait(lk, [&] { return sv->pre_stop || !sv->pre_jobs.empty(); });
            if (sv->pre_jobs.empty()) return;              // stopping, nothing left
            job = sv->pre_jobs.front();
            sv->pre_jobs.pop_front();
        }
        PreDone d;
        d.key = job.key;
        d.tier = job.tier;
        try {
            psp_plan *p = nullptr;
            d.st = psp_plan_create(std::get<0>(job.key), std::get<1>(job.key), std::get<2>(job.key),
                                   job.tier ? PSP_F32 : PSP_F64, &p);
            if (d.st == PSP_OK) {
                d.st = psp_kernel_precompute(p, sv->pre_stream);
                if (d.st != PSP_OK) {
                    d.detail = psp_last_error();
                    psp_plan_destroy(p);
                    p = nullptr;
                }
            } else {
                d.detail = psp_last_error();
            }
            d.plan = p;
        } catch (...) {
            d.st = PSP_ENOMEM;
        }
        {
            std::lock_guard<std::mutex> lk(sv->pre_mu);
            try {
                sv->pre_done.push_back(d);
            } catch (...) {
                if (d.plan) psp_plan_destroy(d.plan);
            }
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->cv_work.notify_one();
        }
    }
}

// finish a request that is still queued (and not done): it leaves the queue
// in the same critical section, so a concurrent cancel cannot finish it twice
static void finish_if_queued(psp_server *sv, uint64_t id, psp_status st);

// scheduler: take over finished precomputes; a failed one finishes the
// queued requests of its (key, tier) with its status
static void collect_precomputes(psp_server *sv) {
    std::vector<PreDone> done;
    {
        std::lock_guard<std::mutex> lk(sv->pre_mu);
        done.swap(sv->pre_done);
    }
    for (auto &d : done) {
        auto &cs = sv->specs[d.key];
        cs.pending[d.tier] = false;
        if (d.st == PSP_OK) {
            cs.plan[d.tier] = d.plan;
            cs.last_use = Clock::now();
            continue;
        }
        if (!cs.plan[0] && !cs.plan[1] && !cs.pending[0] && !cs.pending[1] && cs.bytes) {
            account(sv, -(long)cs.bytes);      // the reservation is given back
            cs.bytes = 0;
        }
        std::vector<uint64_t> ids;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (uint64_t id : sv->queue) {
                const ServeReq &r = sv->reqs[id];
                if (std::make_tuple(r.n, r.h, r.R) == d.key && (r.tier == PSP_F32 ? 1 : 0) == d.tier) ids.push_back(id);
            }
        }
        for (uint64_t id : ids) finish_if_queued(sv, id, d.st);
    }
}

static psp_status take_ws(psp_server *sv, int n, bool f32, PooledWs *out) {
    for (size_t i = 0; i < sv->pool.size(); ++i) {
        if (sv->pool[i].n == n && sv->pool[i].f32 == f32) {
            *out = sv->pool[i];
            sv->pool.erase(sv->pool.begin() + i);
            return PSP_OK;
        }
    }
    PooledWs p;
    p.n = n;
    p.f32 = f32;
    psp_status st = alloc_workspace(n, f32, 0, &p.w);
    if (st != PSP_OK) return st;
    account(sv, (long)p.w.bytes);
    *out = p;
    return PSP_OK;
}

// outcomes of this many completed requests stay available to psp_serve_poll
constexpr size_t kKeepFinished = size_t(1) << 20;

// caller holds sv->mu
static void finish_locked(psp_server *sv, uint64_t id, psp_status st) {
    auto &r = sv->reqs[id];
    r.done = true;
    r.result = st;
    r.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.t_submit).count();
    sv->finished.push_back(id);
    while (sv->finished.size() > kKeepFinished) {
        sv->reqs.erase(sv->finished.front());
        sv->finished.pop_front();
    }
    sv->pending_total--;
    sv->completed++;
    sv->cv_done.notify_all();
}

static void finish(psp_server *sv, uint64_t id, psp_status st) {
    std::lock_guard<std::mutex> lk(sv->mu);
    finish_locked(sv, id, st);
}

static void finish_if_queued(psp_server *sv, uint64_t id, psp_status st) {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto q = std::find(sv->queue.begin(), sv->queue.end(), id);
    if (q == sv->queue.end() || sv->reqs[id].done) return;   // canceled meanwhile
    sv->queue.erase(q);
    finish_locked(sv, id, st);
}

static void retire(psp_server *sv, bool wait) {
    for (auto it = sv->inflight.begin(); it != sv->inflight.end();) {
        hipError_t q = wait ? hipEventSynchronize(it->ev) : hipEventQuery(it->ev);
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        const psp_status st = q == hipSuccess ? PSP_OK : PSP_EHIP;
        for (uint64_t id : it->ids) finish(sv, id, st);
        for (auto &w : it->ws) sv->pool.push_back(w);
        for (auto &k : it->keys) sv->specs[k].users--;
        sv->slots_used -= (int)it->ids.size();
        (void)hipEventDestroy(it->ev);
        it = sv->inflight.erase(it);
    }
}

// One scheduling round: retire finished batches, admit and launch what fits.
// Returns true once the server is stopping and nothing is left.
static bool schedule_round(psp_server *sv) {
    retire(sv, false);
    collect_precomputes(sv);
    // snapshot the queue under the lock: up to the free slots' worth of
    // requests, skipping those whose spectrum is still being precomputed
    // (bounded scan)
    std::vector<std::pair<uint64_t, ServeReq>> cand;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->queue.empty() && sv->inflight.empty()) {
            if (sv->stop) return true;
            sv->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            return false;
        }
        int scanned = 0;
        for (uint64_t id : sv->queue) {
            if ((int)cand.size() + sv->slots_used >= sv->max_slots || ++scanned > 4096) break;
            const ServeReq &r = sv->reqs[id];
            auto sit = sv->specs.find(std::make_tuple(r.n, r.h, r.R));
            if (sit != sv->specs.end() && sit->second.pending[r.tier == PSP_F32 ? 1 : 0]) continue;
            cand.emplace_back(id, r);
        }
    }
    // admit in order; batches per (tier, size class), so that a small
    // request never waits for a large one's completion event
    std::vector<uint64_t> admitted;
    std::vector<SolveArgs> args[kBatchKinds];
    std::vector<uint64_t> ids[kBatchKinds];
    std::vector<PooledWs> wss[kBatchKinds];
    std::vector<SpecKey3> keys[kBatchKinds];
    bool issued = false;
    for (auto &c : cand) {
        const ServeReq &r = c.second;
        const SpecKey3 key = std::make_tuple(r.n, r.h, r.R);
        const bool f32 = r.tier == PSP_F32;
        const int ti = f32 ? 1 : 0;
        CachedSpec &cs = sv->specs[key];
        if (cs.pending[ti]) continue;                 // issued earlier in this round
        if (!cs.plan[ti]) {
            // spectrum-cache miss: reserve the octant (once per key), hand the
            // precompute to its thread; the request stays queued
            const size_t need = cs.bytes ? 0 : spectrum_bytes(r.n);
            if (!make_room(sv, need, &key)) break;    // head of line waits for memory
            if (need) {
                cs.bytes = need;
                account(sv, (long)need);
            }
            cs.pending[ti] = true;
            cs.last_use = Clock::now();
            {
                std::lock_guard<std::mutex> lk(sv->pre_mu);
                sv->pre_jobs.push_back(PreJob{key, ti});
                sv->pre_cv.notify_one();
            }
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->reqs[c.first].missed = true;
            }
            issued = true;
            continue;
        }
        // a pooled workspace of this (n, tier) is taken out of the pool before
        // making room, so that making room cannot evict it; a new one counts
        // against the budget
        PooledWs w;
        bool have_ws = false;
        for (size_t i = 0; i < sv->pool.size(); ++i)
            if (sv->pool[i].n == r.n && sv->pool[i].f32 == f32) {
                w = sv->pool[i];
                sv->pool.erase(sv->pool.begin() + i);
                have_ws = true;
                break;
            }
        if (!make_room(sv, have_ws ? 0 : ws_bytes(r.n, f32), &key)) {
            if (have_ws) sv->pool.push_back(w);
            break;                                    // head of line waits for memory
        }
        psp_status st = PSP_OK;
        if (!have_ws) st = take_ws(sv, r.n, f32, &w);
        admitted.push_back(c.first);
        if (st != PSP_OK) {
            finish_if_queued(sv, c.first, st);
            continue;
        }
        bool missed = false;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            missed = sv->reqs[c.first].missed;
        }
        (missed ? sv->misses : sv->hits)++;
        cs.users++;
        cs.last_use = Clock::now();
        const int t = ti + (r.n > kSmallN ? 2 : 0);
        args[t].push_back(solve_args(cs.plan[ti], w.w, r.rho, r.u));
        ids[t].push_back(c.first);
        wss[t].push_back(w);
        keys[t].push_back(key);
    }
    if (!admitted.empty()) {
        // claim the admitted requests; one canceled (or failed) since the
        // snapshot is no longer queued: drop it from the launch
        std::vector<uint64_t> gone;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (uint64_t id : admitted) {
                auto it = std::find(sv->queue.begin(), sv->queue.end(), id);
                if (it != sv->queue.end())
                    sv->queue.erase(it);
                else
                    gone.push_back(id);
            }
        }
        for (uint64_t id : gone)
            for (int t = 0; t < kBatchKinds; ++t)
                for (size_t i = 0; i < ids[t].size(); ++i)
                    if (ids[t][i] == id) {
                        sv->pool.push_back(wss[t][i]);
                        sv->specs[keys[t][i]].users--;
                        ids[t].erase(ids[t].begin() + i);
                        wss[t].erase(wss[t].begin() + i);
                        keys[t].erase(keys[t].begin() + i);
                        args[t].erase(args[t].begin() + i);
                        break;
                    }
    }
    for (int t = 0; t < kBatchKinds; ++t) {
        if (ids[t].empty()) continue;
        // the stream of this size class with the fewest batches in flight
        std::vector<int> load(sv->streams.size(), 0);
        for (auto &b : sv->inflight) load[b.stream]++;
        const int first = t >= 2 ? kClassStreams : 0;
        const int si = (int)(std::min_element(load.begin() + first, load.begin() + first + kClassStreams) -
                             load.begin());
        hipStream_t st = sv->streams[si];
        Batch b;
        b.stream = si;
        hipError_t e = launch_batch((int)args[t].size(), args[t].data(), st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b.ev, st);
        if (e != hipSuccess) {
            for (uint64_t id : ids[t]) finish(sv, id, PSP_EHIP);
            for (auto &w : wss[t]) sv->pool.push_back(w);
            for (auto &k : keys[t]) sv->specs[k].users--;
            continue;
        }
        b.ids = ids[t];
        b.ws = wss[t];
        b.keys = keys[t];
        sv->slots_used += (int)b.ids.size();
        sv->inflight.push_back(std::move(b));
    }
    if (admitted.empty() && !issued) {
        // nothing admitted: wait for a completion or a new request
        if (!sv->inflight.empty()) {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
    return false;
}

// A host allocation failed inside a round: the requests that round had taken
// off the queue but not launched are finished with PSP_ENOMEM, so that no
// caller waits for them; queued and in-flight requests carry on.  (Their
// workspaces and spectrum references of that round are not returned.)
static void fail_unlaunched(psp_server *sv) noexcept {
    try {
        std::vector<uint64_t> live;
        for (auto &b : sv->inflight) live.insert(live.end(), b.ids.begin(), b.ids.end());
        std::lock_guard<std::mutex> lk(sv->mu);
        std::vector<uint64_t> lost;
        for (auto &kv : sv->reqs) {
            if (kv.second.done) continue;
            if (std::find(sv->queue.begin(), sv->queue.end(), kv.first) != sv->queue.end()) continue;
            if (std::find(live.begin(), live.end(), kv.first) != live.end()) continue;
            lost.push_back(kv.first);
        }
        for (uint64_t id : lost) finish_locked(sv, id, PSP_ENOMEM);
    } catch (...) {
    }
}

static void scheduler(psp_server *sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        bool stop = false;
        try {
            stop = schedule_round(sv);
        } catch (...) {
            fail_unlaunched(sv);
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
        }
        if (stop) break;
    }
    try {
        retire(sv, true);
    } catch (...) {
    }
}

}  // namespace psp

extern "C" {

psp_status psp_serve_create(size_t hbm_budget_bytes, int max_slots, psp_server **out) {
    return guarded([&]() -> psp_status {
        if (!out) return fail(PSP_EINVAL, "out is NULL");
        *out = nullptr;
        if (hbm_budget_bytes == 0 || max_slots < 1) return fail(PSP_EINVAL, "budget and max_slots must be positive");
        psp_server *sv = new (std::nothrow) psp_server;
        if (!sv) return fail(PSP_ENOMEM, "host allocation failed");
        sv->budget = hbm_budget_bytes;
        sv->max_slots = max_slots;
        if (hipGetDevice(&sv->device) != hipSuccess) {
            delete sv;
            return fail(PSP_EHIP, "hipGetDevice failed");
        }
        for (int i = 0; i < 2 * kClassStreams + 1; ++i) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
                for (auto x : sv->streams) (void)hipStreamDestroy(x);
                if (sv->pre_stream) (void)hipStreamDestroy(sv->pre_stream);
                delete sv;
                return fail(PSP_EHIP, "hipStreamCreate failed");
            }
            if (i < 2 * kClassStreams)
                sv->streams.push_back(s);
            else
                sv->pre_stream = s;
        }
        sv->pre_thread = std::thread(precompute_worker, sv);
        sv->sched = std::thread(scheduler, sv);
        *out = sv;
        return PSP_OK;
    });
}

psp_status psp_serve_submit(psp_server *sv, int n, double h, int R, psp_dtype tier, const void *rho_dev,
                            void *u_dev, uint64_t *ticket) {
    return guarded([&]() -> psp_status {
        if (!sv || !rho_dev || !u_dev || !ticket) return fail(PSP_EINVAL, "NULL argument");
        if (tier != PSP_F64 && tier != PSP_F32) return fail(PSP_EINVAL, "unknown tier");
        const double half = (double)n * h;
        psp_status st = check_create(n, h, R, 1e-4 * half, std::sqrt(3.0) * half);
        if (st != PSP_OK) return st;
        if (spectrum_bytes(n) + ws_bytes(n, tier == PSP_F32) > sv->budget)
            return fail(PSP_ENOMEM, "request footprint exceeds the whole budget");
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->queue.size() >= 65536) return fail(PSP_EBUSY, "queue full");
        ServeReq r;
        r.n = n;
        r.h = h;
        r.R = R;
        r.tier = tier;
        r.rho = rho_dev;
        r.u = u_dev;
        r.t_submit = Clock::now();
        const uint64_t id = sv->next_id++;
        sv->reqs.emplace(id, r);
        sv->queue.push_back(id);
        sv->pending_total++;
        *ticket = id;
        sv->cv_work.notify_one();
        return PSP_OK;
    });
}

psp_status psp_serve_cancel(psp_server *sv, uint64_t ticket) {
    return guarded([&]() -> psp_status {
        if (!sv) return fail(PSP_EINVAL, "server is NULL");
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end() || it->second.done)
            return fail(PSP_EINVAL, "unknown or finished ticket %llu", (unsigned long long)ticket);
        auto q = std::find(sv->queue.begin(), sv->queue.end(), ticket);
        if (q == sv->queue.end()) return fail(PSP_EBUSY, "request %llu is on the device", (unsigned long long)ticket);
        sv->queue.erase(q);
        finish_locked(sv, ticket, PSP_ECANCELED);
        return PSP_OK;
    });
}

psp_status psp_serve_poll(psp_server *sv, uint64_t ticket, int *done, psp_status *result, double *latency_ms) {
    return guarded([&]() -> psp_status {
        if (!sv) return fail(PSP_EINVAL, "server is NULL");
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end())
            return fail(PSP_EINVAL, "unknown or expired ticket %llu", (unsigned long long)ticket);
        if (done) *done = it->second.done ? 1 : 0;
        if (result) *result = it->second.result;
        if (latency_ms) *latency_ms = it->second.latency_ms;
        return PSP_OK;
    });
}

psp_status psp_serve_drain(psp_server *sv) {
    return guarded([&]() -> psp_status {
        if (!sv) return fail(PSP_EINVAL, "server is NULL");
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->pending_total == 0; });
        return PSP_OK;
    });
}

psp_status psp_serve_stats(psp_server *sv, size_t *bytes_in_use, size_t *bytes_peak, uint64_t *completed,
                           uint64_t *cache_hits, uint64_t *cache_misses) {
    return guarded([&]() -> psp_status {
        if (!sv) return fail(PSP_EINVAL, "server is NULL");
        if (bytes_in_use) *bytes_in_use = sv->bytes_in_use.load();
        if (bytes_peak) *bytes_peak = sv->bytes_peak.load();
        if (completed) *completed = sv->completed.load();
        if (cache_hits) *cache_hits = sv->hits.load();
        if (cache_misses) *cache_misses = sv->misses.load();
        return PSP_OK;
    });
}

void psp_serve_destroy(psp_server *sv) {
    try {
        if (!sv) return;
        psp_serve_drain(sv);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
            sv->cv_work.notify_all();
        }
        sv->sched.join();
        {
            std::lock_guard<std::mutex> lk(sv->pre_mu);
            sv->pre_stop = true;
            sv->pre_cv.notify_all();
        }
        sv->pre_thread.join();
        for (auto &d : sv->pre_done)
            if (d.plan) psp_plan_destroy(d.plan);
        for (auto &w : sv->pool) free_ws(sv, w);
        for (auto &kv : sv->specs)
            for (int t = 0; t < 2; ++t) psp_plan_destroy(kv.second.plan[t]);
        for (auto s : sv->streams) (void)hipStreamDestroy(s);
        (void)hipStreamDestroy(sv->pre_stream);
        delete sv;
    } catch (...) {
    }
}

}  // extern "C"
