// batched.hip - many independent solves on one stream, grouped by padded
// length and launch shape: one launch per pass per distinct (n, shape).
// Each solve has its own workspace (one chunk of all k3 tiles) and its
// pointers in a device job table that the pass kernels index with
// blockIdx.y; the table is staged
// through pinned host memory.  Every solve runs the same kernels on the same
// data as a single psp_solve, so the results are bitwise equal.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "host_common.hpp"

namespace psp {

struct Staging {
    Job *h = nullptr;      // pinned host copy of the table
    Job *d = nullptr;      // device table
    size_t cap = 0;
    hipEvent_t uploaded = nullptr;   // the last upload has read the pinned copy
};

struct StreamBatch {
    Staging stage;
    std::map<std::pair<int, bool>, std::vector<Workspace>> ws;   // (n, f32) -> pool
};

static std::mutex g_batch_mu;
static std::map<std::pair<int, hipStream_t>, StreamBatch> g_batch;   // (device, stream)

static psp_status stage_table(Staging &S, const std::vector<Job> &jobs, hipStream_t st, Job **d_out) {
    if (S.uploaded) {
        hipError_t e = hipEventSynchronize(S.uploaded);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(batch table)");
    }
    if (S.cap < jobs.size()) {
        if (S.h) (void)hipHostFree(S.h);
        if (S.d) (void)hipFree(S.d);
        S.h = nullptr;
        S.d = nullptr;
        S.cap = 0;
        const size_t cap = std::max<size_t>(jobs.size(), 64);
        if (hipHostMalloc((void **)&S.h, cap * sizeof(Job)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(PSP_ENOMEM, "pinned batch table allocation failed");
        }
        if (hipMalloc((void **)&S.d, cap * sizeof(Job)) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(S.h);
            S.h = nullptr;
            return fail(PSP_ENOMEM, "batch table allocation failed");
        }
        S.cap = cap;
    }
    if (!S.uploaded && hipEventCreateWithFlags(&S.uploaded, hipEventDisableTiming) != hipSuccess)
        return fail(PSP_EHIP, "hipEventCreate failed");
    std::memcpy(S.h, jobs.data(), jobs.size() * sizeof(Job));
    hipError_t e = hipMemcpyAsync(S.d, S.h, jobs.size() * sizeof(Job), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(S.uploaded, st);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    *d_out = S.d;
    return PSP_OK;
}

// launch the grouped passes for jobs already holding workspaces
static psp_status launch_jobs(StreamBatch &B, const std::vector<Job> &jobs, const std::vector<int> &ns,
                              const std::vector<Shape> &shapes, bool f32, const std::vector<const Twiddles *> &tws,
                              hipStream_t st) {
    // order by (n, shape) so that each group is a contiguous slice of the table
    std::vector<int> order(jobs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (ns[a] != ns[b]) return ns[a] < ns[b];
        return shapes[a] < shapes[b];
    });
    std::vector<Job> sorted(jobs.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = jobs[order[i]];
    Job *d = nullptr;
    psp_status rs = stage_table(B.stage, sorted, st, &d);
    if (rs != PSP_OK) return rs;
    size_t i = 0;
    while (i < order.size()) {
        size_t j = i;
        while (j < order.size() && ns[order[j]] == ns[order[i]] && shapes[order[j]] == shapes[order[i]]) ++j;
        const Twiddles *tw = tws[order[i]];
        hipError_t e = launch_group(ns[order[i]], f32, shapes[order[i]], d + i, (int)(j - i),
                                    f32 ? tw->hi32 : tw->w64, f32 ? tw->lo32 : nullptr, st);
        if (e != hipSuccess) return hip_fail(e, "batched pass launch");
        i = j;
    }
    return PSP_OK;
}

// caller holds g_batch_mu; the pointers stay valid until the pool grows
static psp_status batch_workspaces(StreamBatch &B, const std::vector<int> &ns, bool f32,
                                   std::vector<Workspace *> &out) {
    // grow every pool to the count this batch needs first: pointers into a
    // pool are taken only after it has stopped growing
    std::map<int, size_t> need;
    for (int n : ns) need[n]++;
    for (const auto &kv : need) {
        auto &pool = B.ws[{kv.first, f32}];
        while (pool.size() < kv.second) {
            Workspace w;
            psp_status rs = alloc_workspace(kv.first, f32, 0, &w);
            if (rs != PSP_OK) return rs;
            pool.push_back(w);
        }
    }
    std::map<int, size_t> used;
    out.clear();
    for (int n : ns) out.push_back(&B.ws[{n, f32}][used[n]++]);
    return PSP_OK;
}

// serving: jobs whose workspaces the caller owns (one chunk of all tiles)
hipError_t launch_batch(int count, const SolveArgs *args, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<Job> jobs(count);
    std::vector<int> ns(count);
    std::vector<Shape> shapes(count);
    std::vector<const Twiddles *> tws(count);
    for (int i = 0; i < count; ++i) {
        const SolveArgs &a = args[i];
        jobs[i] = Job{a.rho, a.u, a.X, a.A, a.mult, nullptr, nullptr};
        ns[i] = a.n;
        shapes[i] = a.shape;
        if (get_twiddles(dev, 2 * a.n, &tws[i]) != PSP_OK) return hipErrorOutOfMemory;
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    psp_status rs = launch_jobs(g_batch[{dev, st}], jobs, ns, shapes, args[0].f32, tws, st);
    return rs == PSP_OK ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace psp

using namespace psp;

extern "C" psp_status psp_solve_batched(int count, psp_plan *const *plans, const void *const *rho_dev,
                                        void *const *u_dev, void *stream) {
    if (count < 0 || (count > 0 && (!plans || !rho_dev || !u_dev))) return fail(PSP_EINVAL, "bad batch arguments");
    if (count == 0) return PSP_OK;
    if (count > 65535) return fail(PSP_EINVAL, "at most 65535 solves per batch");
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !rho_dev[i] || !u_dev[i]) return fail(PSP_EINVAL, "NULL entry %d in batch", i);
        if (!plans[i]->precomputed) return fail(PSP_ESTATE, "batch entry %d not precomputed", i);
        if (plans[i]->dtype != plans[0]->dtype) return fail(PSP_EINVAL, "batch mixes dtypes");
        if (plans[i]->device != plans[0]->device) return fail(PSP_EINVAL, "batch mixes devices");
        if (rho_dev[i] == u_dev[i]) return fail(PSP_EINVAL, "entry %d: rho and u must not alias", i);
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plans[0]->device)
        return fail(PSP_EINVAL, "plans were precomputed on device %d, current is %d", plans[0]->device, dev);
    hipStream_t st = (hipStream_t)stream;
    const bool f32 = plans[0]->dtype == PSP_F32;
    std::vector<int> ns(count);
    for (int i = 0; i < count; ++i) ns[i] = plans[i]->n;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    StreamBatch &B = g_batch[{dev, st}];
    std::vector<Workspace *> ws;
    psp_status rs = batch_workspaces(B, ns, f32, ws);
    if (rs != PSP_OK) return rs;
    std::vector<Job> jobs(count);
    std::vector<Shape> shapes(count);
    std::vector<const Twiddles *> tws(count);
    for (int i = 0; i < count; ++i) {
        jobs[i] = Job{rho_dev[i], u_dev[i], ws[i]->X, ws[i]->A, plans[i]->spec->mult, nullptr, nullptr};
        shapes[i] = plans[i]->shape;
        tws[i] = plans[i]->tw;
    }
    return launch_jobs(B, jobs, ns, shapes, f32, tws, st);
}
