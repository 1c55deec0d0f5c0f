// graph.cpp - solves captured as HIP graphs.  A graph owns its workspaces
// and (for batches) its device job table, written before capture, so its
// replays read nothing from library state that later calls may change.
#include <algorithm>
#include <vector>

#include "host_common.hpp"

struct psp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<psp::Workspace> ws;
    unsigned char *table = nullptr;   // device batch image
    int device = -1;
};

namespace psp {

static void graph_free(psp_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (auto &w : g->ws) free_workspace(&w);
    if (g->table) (void)hipFree(g->table);
    delete g;
}

// capture `record` on a private stream forked from `stream`
template <typename F>
static psp_status capture(psp_graph *g, hipStream_t stream, F record) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(PSP_EHIP, "hipStreamCreate");
    // everything the graph reads was written on `stream` before this call
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    hipError_t le = record(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return PSP_OK;
}

}  // namespace psp

using namespace psp;

extern "C" {

psp_status psp_graph_capture(const psp_plan *p, const void *rho_dev, void *u_dev, void *stream, psp_graph **out) {
    return guarded([&]() -> psp_status {
        if (!out) return fail(PSP_EINVAL, "out is NULL");
        *out = nullptr;
        if (!p || !rho_dev || !u_dev) return fail(PSP_EINVAL, "NULL argument");
        if (!p->precomputed) return fail(PSP_ESTATE, "capture before psp_kernel_precompute");
        if (rho_dev == u_dev) return fail(PSP_EINVAL, "rho and u must not alias");
        psp_graph *g = new (std::nothrow) psp_graph;
        if (!g) return fail(PSP_ENOMEM, "host allocation failed");
        g->device = p->device;
        g->ws.resize(1);
        psp_status rs = p->grid ? alloc_workspace_dims(Dims{p->ns[0], p->ns[1], p->ns[2]}, p->dtype == PSP_F32, &g->ws[0])
                                : alloc_workspace(p->n, p->dtype == PSP_F32, 0, &g->ws[0]);
        if (rs != PSP_OK) {
            g->ws.clear();
            graph_free(g);
            return rs;
        }
        SolveArgs a = solve_args(p, g->ws[0], rho_dev, u_dev);
        a.chunk_tiles = 0;
        rs = capture(g, (hipStream_t)stream, [&](hipStream_t cs) { return launch_solve(a, cs); });
        if (rs != PSP_OK) {
            graph_free(g);
            return rs;
        }
        *out = g;
        return PSP_OK;
    });
}

psp_status psp_graph_capture_batched(int count, const psp_plan *const *plans, const void *const *rho_dev,
                                     void *const *u_dev, void *stream, psp_graph **out) {
    return guarded([&]() -> psp_status {
        if (!out) return fail(PSP_EINVAL, "out is NULL");
        *out = nullptr;
        if (count < 1 || count > 65535 || !plans || !rho_dev || !u_dev) return fail(PSP_EINVAL, "bad batch arguments");
        for (int i = 0; i < count; ++i) {
            if (!plans[i] || !rho_dev[i] || !u_dev[i]) return fail(PSP_EINVAL, "NULL entry %d in batch", i);
            if (!plans[i]->precomputed) return fail(PSP_ESTATE, "batch entry %d not precomputed", i);
            if (plans[i]->dtype != plans[0]->dtype) return fail(PSP_EINVAL, "batch mixes dtypes");
        }
        const bool f32 = plans[0]->dtype == PSP_F32;
        psp_graph *g = new (std::nothrow) psp_graph;
        if (!g) return fail(PSP_ENOMEM, "host allocation failed");
        g->device = plans[0]->device;
        g->ws.resize(count);
        // cubes go through the batch image; grids with unequal counts follow,
        // each with its own per-axis launch sequence
        std::vector<BatchMember> m;
        std::vector<SolveArgs> grid_args;
        for (int i = 0; i < count; ++i) {
            const psp_plan *p = plans[i];
            psp_status rs = p->grid ? alloc_workspace_dims(Dims{p->ns[0], p->ns[1], p->ns[2]}, f32, &g->ws[i])
                                    : alloc_workspace(p->n, f32, 0, &g->ws[i]);
            if (rs != PSP_OK) {
                g->ws.resize(i);
                graph_free(g);
                return rs;
            }
            if (p->grid) {
                grid_args.push_back(solve_args(p, g->ws[i], rho_dev[i], u_dev[i]));
                continue;
            }
            BatchMember b;
            b.job = Job{rho_dev[i], u_dev[i], g->ws[i].X, g->ws[i].A, p->spec->mult, nullptr, nullptr};
            b.n = p->n;
            b.shape = p->shape;
            b.tw64 = p->tw->w64;
            m.push_back(b);
        }
        // the batch image is written once, before capture; each replay clears
        // the persistent counters with a kernel (no memset node in the graph)
        BatchImage img;
        if (!m.empty()) {
            if (persist_prepare() != hipSuccess) {
                (void)hipGetLastError();
                graph_free(g);
                return fail(PSP_EHIP, "occupancy query failed");
            }
            std::vector<unsigned char> host;
            if (hipMalloc((void **)&g->table, batch_image_bytes(m)) != hipSuccess) {
                (void)hipGetLastError();
                g->table = nullptr;
                graph_free(g);
                return fail(PSP_ENOMEM, "graph batch table allocation failed");
            }
            build_batch_image(m, f32, g->table, &img, host);
            if (hipMemcpy(g->table, host.data(), img.bytes, hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipGetLastError();
                graph_free(g);
                return fail(PSP_EHIP, "graph batch table upload failed");
            }
        }
        psp_status rs = capture(g, (hipStream_t)stream, [&](hipStream_t cs) -> hipError_t {
            hipError_t e = m.empty() ? hipSuccess : launch_batch_image(m, img, f32, g->table, true, cs);
            for (const SolveArgs &a : grid_args) {
                if (e != hipSuccess) break;
                e = launch_solve(a, cs);
            }
            return e;
        });
        if (rs != PSP_OK) {
            graph_free(g);
            return rs;
        }
        *out = g;
        return PSP_OK;
    });
}

psp_status psp_graph_launch(psp_graph *g, void *stream) {
    return guarded([&]() -> psp_status {
        if (!g || !g->exec) return fail(PSP_EINVAL, "graph is NULL");
        hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return PSP_OK;
    });
}

void psp_graph_destroy(psp_graph *g) { graph_free(g); }

}  // extern "C"
