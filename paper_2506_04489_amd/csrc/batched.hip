// batched.hip - many independent solves on one stream.  By default solves
// are grouped by (n, shape) with one launch per pass per group.  In the
// persistent batch mode, solves with padded length 2n <= 256 run through the
// persistent pass kernels instead (one launch per pass for all of them, work
// items from atomic counters) and only larger ones (and those with a radix-16
// plan) are grouped.  Each solve
// has its own workspace (one chunk of all k3 tiles).  The batch image
// (persistent header, job table, item offsets and the grouped job table) is
// built on the host and uploaded in one copy through pinned memory.  Grids
// with unequal point counts per axis run after the cubes, each with its own
// per-axis launch sequence, one workspace per distinct grid.  Every solve
// runs the same arithmetic as a single psp_solve, so the results are bitwise
// equal.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "host_common.hpp"

namespace psp {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// batch mode (psp_set_batch_mode): 0 grouped launches, 1 persistent kernels
// for 2n <= 256, 2 the same kernels with one workgroup per item.  Measured on
// MI355X for the 64-mixture batch (n = 32..128, FP64): grouped 29.9k
// solves/s, flat 25.6k, persistent 19.0k, one solve at a time 21.9k (each
// persistent workgroup runs its items one after another and exposes every
// item's load latency); so grouped launches are the default.
static std::atomic<int> g_batch_mode{0};
static bool persistent_enabled() { return g_batch_mode.load() != 0; }

static void image_layout(const std::vector<BatchMember> &m, BatchImage *img) {
    img->persist.clear();
    img->grouped.clear();
    const bool pers = persistent_enabled();
    for (int i = 0; i < (int)m.size(); ++i) {
        // the persistent kernels size their LDS for radices up to 8: up to
        // 2n = PB_MAX_N only plan 2 has a larger one (persist.hpp checks
        // plans 0 and 1 at compile time)
        bool r16 = false;
        for (int p = 0; p < kPasses; ++p) r16 |= m[i].shape.plan[p] == 2;
        // and exist for the lengths whose threads per column divide their
        // workgroup (persist_tpc is 0 for the others)
        const bool built = 2 * m[i].n <= PB_MAX_N && persist_tpc(2 * m[i].n, 0) > 0;
        (pers && !r16 && built ? img->persist : img->grouped).push_back(i);
    }
    // persistent jobs by decreasing n (the largest items are taken first);
    // grouped jobs by (n, shape) so that each group is a contiguous slice
    std::stable_sort(img->persist.begin(), img->persist.end(), [&](int a, int b) { return m[a].n > m[b].n; });
    std::stable_sort(img->grouped.begin(), img->grouped.end(), [&](int a, int b) {
        if (m[a].n != m[b].n) return m[a].n < m[b].n;
        return m[a].shape < m[b].shape;
    });
    const size_t k = img->persist.size();
    img->hdr_off = 0;
    img->jobs_off = align256(sizeof(PBatch));
    img->start_off = align256(img->jobs_off + k * sizeof(PJob));
    img->group_off = align256(img->start_off + (size_t)kPasses * (k + 1) * sizeof(int));
    img->bytes = align256(img->group_off + img->grouped.size() * sizeof(Job));
}

// items of pass p for one solve on the persistent path
static int persist_items(int n, int pv, int p) {
    const int N = 2 * n, tpc = persist_tpc(N, pv);
    const long w = PB_THREADS / tpc;
    long count;
    if (p == 0 || p == 4) count = (long)n * n / 2;
    else if (p == 2) count = (long)N * (n + 1);
    else count = (long)n * (n + 1);
    return (int)((count + w - 1) / w);
}

size_t batch_image_bytes(const std::vector<BatchMember> &m) {
    BatchImage img;
    image_layout(m, &img);
    return img.bytes;
}

void build_batch_image(const std::vector<BatchMember> &m, bool f32, unsigned char *dev_base, BatchImage *img,
                       std::vector<unsigned char> &host) {
    image_layout(m, img);
    img->flat = g_batch_mode.load() == 2;
    host.assign(img->bytes, 0);
    const int k = (int)img->persist.size();
    PBatch hdr{};
    hdr.njobs = k;
    hdr.jobs = (const PJob *)(dev_base + img->jobs_off);
    hdr.start = (const int *)(dev_base + img->start_off);
    PJob *jobs = (PJob *)(host.data() + img->jobs_off);
    int *start = (int *)(host.data() + img->start_off);
    for (int p = 0; p < kPasses; ++p) {
        int acc = 0;
        for (int j = 0; j < k; ++j) {
            start[p * (k + 1) + j] = acc;
            const BatchMember &b = m[img->persist[j]];
            acc += persist_items(b.n, b.shape.plan[p], p);
        }
        start[p * (k + 1) + k] = acc;
        hdr.total[p] = acc;
        img->total[p] = acc;
    }
    const int LW = strided_width(f32);
    for (int j = 0; j < k; ++j) {
        const BatchMember &b = m[img->persist[j]];
        PJob &pj = jobs[j];
        pj.rho = b.job.rho;
        pj.u = b.job.u;
        pj.X = b.job.X;
        pj.A = b.job.A;
        pj.mult = b.job.mult;
        pj.tw64 = b.tw64;
        pj.N = 2 * b.n;
        pj.P = pitch_for(b.n);
        pj.pa = ((b.n + 1 + LW - 1) / LW) * LW;   // one chunk holding all tiles
        pj.plane = (long long)a_plane(b.n, b.n, pj.pa, f32 ? 8 : 16);
        for (int p = 0; p < kPasses; ++p) pj.pv[p] = b.shape.plan[p];
    }
    std::memcpy(host.data() + img->hdr_off, &hdr, sizeof(hdr));
    Job *gt = (Job *)(host.data() + img->group_off);
    for (size_t i = 0; i < img->grouped.size(); ++i) gt[i] = m[img->grouped[i]].job;
}

hipError_t launch_batch_image(const std::vector<BatchMember> &m, const BatchImage &img, bool f32,
                              unsigned char *dev_base, bool reset, hipStream_t st) {
    if (!img.persist.empty()) {
        PBatch *hdr = (PBatch *)(dev_base + img.hdr_off);
        hipError_t e = img.flat ? flat_launch(f32, hdr, img.total, st) : persist_launch(f32, hdr, img.total, reset, st);
        if (e != hipSuccess) return e;
    }
    const std::vector<int> &g = img.grouped;
    size_t i = 0;
    while (i < g.size()) {
        size_t j = i;
        const BatchMember &b = m[g[i]];
        while (j < g.size() && m[g[j]].n == b.n && m[g[j]].shape == b.shape) ++j;
        hipError_t e = launch_group(b.n, f32, b.shape, (const Job *)(dev_base + img.group_off) + i, (int)(j - i),
                                    b.tw64, st);
        if (e != hipSuccess) return e;
        i = j;
    }
    return hipSuccess;
}

// A stream's batch tables go up through a ring of kStageSlots slots, each a
// pinned host copy and the device image it is copied to.  A slot's host copy
// is rewritten only once its previous upload has read it (its event); its
// device image is overwritten by a copy that runs, in stream order, after the
// kernels that read it.  With a single slot, every batch waited on the host
// for the stream to reach the previous batch's upload, i.e. for all work
// queued before that: a serving loop then stalled for milliseconds behind
// large solves.  The host now blocks only when kStageSlots uploads are still
// queued on the stream.
struct StageSlot {
    unsigned char *h = nullptr;   // pinned host copy of the image
    unsigned char *d = nullptr;   // device image
    size_t cap = 0;
    hipEvent_t uploaded = nullptr;   // the last upload from this slot has read h
    bool used = false;
};
constexpr int kStageSlots = 8;
struct Staging {
    StageSlot slot[kStageSlots];
    int next = 0;
};

struct StreamBatch {
    Staging stage;
    std::map<std::pair<int, bool>, std::vector<Workspace>> ws;   // (n, f32) -> pool
    // grids: one workspace per (n1, n2, n3, f32); their solves run one after
    // another on the stream, so they can share it
    std::map<std::pair<std::vector<int>, bool>, Workspace> grid_ws;
};

static std::mutex g_batch_mu;
static std::map<std::pair<int, hipStream_t>, StreamBatch> g_batch;   // (device, stream)

// build, upload through pinned memory and launch
static psp_status run_batch(Staging &ring, const std::vector<BatchMember> &m, bool f32, hipStream_t st) {
    StageSlot &S = ring.slot[ring.next];
    ring.next = (ring.next + 1) % kStageSlots;
    if (S.used) {
        hipError_t e = hipEventSynchronize(S.uploaded);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(batch table)");
    }
    const size_t need = batch_image_bytes(m);
    if (S.cap < need) {
        if (S.h) (void)hipHostFree(S.h);
        if (S.d) (void)hipFree(S.d);
        S.h = S.d = nullptr;
        S.cap = 0;
        const size_t cap = std::max<size_t>(need, 64 * 1024);
        if (hipHostMalloc((void **)&S.h, cap) != hipSuccess) {
            (void)hipGetLastError();
            S.h = nullptr;
            return fail(PSP_ENOMEM, "pinned batch table allocation failed");
        }
        if (hipMalloc((void **)&S.d, cap) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(S.h);
            S.h = S.d = nullptr;
            return fail(PSP_ENOMEM, "batch table allocation failed");
        }
        S.cap = cap;
    }
    if (!S.uploaded && hipEventCreateWithFlags(&S.uploaded, hipEventDisableTiming) != hipSuccess)
        return fail(PSP_EHIP, "hipEventCreate failed");
    BatchImage img;
    std::vector<unsigned char> host;
    build_batch_image(m, f32, S.d, &img, host);
    std::memcpy(S.h, host.data(), img.bytes);
    // the upload also clears the persistent counters
    hipError_t e = hipMemcpyAsync(S.d, S.h, img.bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(S.uploaded, st);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    S.used = true;
    e = launch_batch_image(m, img, f32, S.d, false, st);
    if (e != hipSuccess) return hip_fail(e, "batched pass launch");
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
    std::vector<BatchMember> m(count);
    for (int i = 0; i < count; ++i) {
        const SolveArgs &a = args[i];
        m[i].job = Job{a.rho, a.u, a.X, a.A, a.mult, nullptr, nullptr};
        m[i].n = a.n;
        m[i].shape = a.shape;
        m[i].tw64 = a.tw64;
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    psp_status rs = run_batch(g_batch[{dev, st}].stage, m, args[0].f32, st);
    return rs == PSP_OK ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace psp

using namespace psp;

extern "C" psp_status psp_set_batch_mode(int mode) {
    return guarded([&]() -> psp_status {
        if (mode < 0 || mode > 2) return fail(PSP_EINVAL, "batch mode must be 0, 1 or 2 (got %d)", mode);
        g_batch_mode.store(mode);
        return PSP_OK;
    });
}

extern "C" psp_status psp_solve_batched(int count, const psp_plan *const *plans, const void *const *rho_dev,
                                        void *const *u_dev, void *stream) {
    return guarded([&]() -> psp_status {
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
        std::vector<int> cube, grid;
        for (int i = 0; i < count; ++i) (plans[i]->grid ? grid : cube).push_back(i);
        std::lock_guard<std::mutex> lk(g_batch_mu);
        StreamBatch &B = g_batch[{dev, st}];
        // grid workspaces first: an allocation failure leaves nothing enqueued
        std::vector<Workspace *> gws;
        for (int i : grid) {
            const psp_plan *p = plans[i];
            auto key = std::make_pair(std::vector<int>{p->ns[0], p->ns[1], p->ns[2]}, f32);
            auto it = B.grid_ws.find(key);
            if (it == B.grid_ws.end()) {
                Workspace w;
                psp_status rs = alloc_workspace_dims(Dims{p->ns[0], p->ns[1], p->ns[2]}, f32, &w);
                if (rs != PSP_OK) return rs;
                it = B.grid_ws.emplace(key, w).first;
            }
            gws.push_back(&it->second);
        }
        if (!cube.empty()) {
            std::vector<int> ns;
            for (int i : cube) ns.push_back(plans[i]->n);
            std::vector<Workspace *> ws;
            psp_status rs = batch_workspaces(B, ns, f32, ws);
            if (rs != PSP_OK) return rs;
            std::vector<BatchMember> m(cube.size());
            for (size_t j = 0; j < cube.size(); ++j) {
                const int i = cube[j];
                m[j].job = Job{rho_dev[i], u_dev[i], ws[j]->X, ws[j]->A, plans[i]->spec->mult, nullptr, nullptr};
                m[j].n = plans[i]->n;
                m[j].shape = plans[i]->shape;
                m[j].tw64 = plans[i]->tw->w64;
            }
            rs = run_batch(B.stage, m, f32, st);
            if (rs != PSP_OK) return rs;
        }
        for (size_t j = 0; j < grid.size(); ++j) {
            const int i = grid[j];
            const hipError_t e = launch_solve(solve_args(plans[i], *gws[j], rho_dev[i], u_dev[i]), st);
            if (e != hipSuccess) return hip_fail(e, "batched grid solve");
        }
        return PSP_OK;
    });
}
