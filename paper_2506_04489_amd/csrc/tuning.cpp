// tuning.cpp - launch shapes of the passes: per-plan setting, the
// process-wide tuning table, and the autotuner that measures every
// (radix plan, tile) candidate of every pass with HIP events.
#include <algorithm>
#include <cfloat>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "host_common.hpp"

namespace psp {

static std::mutex g_tune_mu;
static std::map<std::pair<int, bool>, Shape> g_tune;   // (n, f32) -> shape

Shape tuned_shape(int n, bool f32) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({n, f32});
    return it == g_tune.end() ? Shape{} : it->second;
}

static psp_status shape_from(int n, const int *plan, const int *tile, Shape *out) {
    if (!plan || !tile) return fail(PSP_EINVAL, "NULL shape array");
    Shape s;
    for (int i = 0; i < kPasses; ++i) {
        s.plan[i] = plan[i];
        s.tile[i] = tile[i];
    }
    if (!shape_valid(n, s)) return fail(PSP_EINVAL, "shape out of range for n = %d", n);
    *out = s;
    return PSP_OK;
}

static void shape_to(const Shape &s, int *plan, int *tile) {
    for (int i = 0; i < kPasses; ++i) {
        if (plan) plan[i] = s.plan[i];
        if (tile) tile[i] = s.tile[i];
    }
}

// one timing input: values in [-1, 1) from an integer hash of the index,
// dense like measured data (all-zero input draws less power and so times
// the arithmetic-heavy candidates too kindly)
template <typename T>
__global__ void k_fill_hash(T *p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t x = (uint32_t)i * 2654435761u + 0x9e3779b9u;
        x ^= x >> 16;
        x *= 0x7feb352du;
        x ^= x >> 15;
        x *= 0x846ca68bu;
        x ^= x >> 16;
        p[i] = T((double)x * (2.0 / 4294967296.0) - 1.0);
    }
}

// the other timing input: a smooth density of compact support, the C-infinity
// bump exp(-1/(1 - r^2/0.36)) for r < 0.6 on [-1, 1)^3 (zero on 97% of the
// grid, the kind of input the solver is meant for); its near-zero
// intermediates draw less power than pseudo-random values, and the order of
// near candidates differs between the two
template <typename T>
__global__ void k_fill_bump(T *p, int n) {
    const size_t count = (size_t)n * n * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const int i3 = (int)(i % n), i2 = (int)((i / n) % n), i1 = (int)(i / ((size_t)n * n));
        const double x = -1.0 + 2.0 * i1 / n, y = -1.0 + 2.0 * i2 / n, z = -1.0 + 2.0 * i3 / n;
        const double q = (x * x + y * y + z * z) / 0.36;
        p[i] = q < 1.0 ? T(exp(-1.0 / (1.0 - q))) : T(0);
    }
}

// candidates (radix plan, tile) of pass i for size n
static std::vector<std::pair<int, int>> candidates(int n, int i) {
    std::vector<std::pair<int, int>> c;
    for (int pl = 0; pl < kMaxPlans; ++pl)
        if (plan_exists(2 * n, pl))
            for (int tl = 0; tl < kTileChoices[i]; ++tl) c.push_back({pl, tl});
    return c;
}

}  // namespace psp

using namespace psp;

extern "C" {

psp_status psp_plan_set_shape(psp_plan *p, const int *plan, const int *tile) {
    return guarded([&]() -> psp_status {
        if (!p) return fail(PSP_EINVAL, "plan is NULL");
        if (p->grid) return fail(PSP_EUNSUPPORTED, "launch shapes of a plan with unequal point counts come from the table");
        Shape s;
        psp_status rs = shape_from(p->n, plan, tile, &s);
        if (rs != PSP_OK) return rs;
        std::lock_guard<std::mutex> lk(p->mu);
        p->shape = s;
        return PSP_OK;
    });
}

psp_status psp_plan_get_shape(const psp_plan *p, int *plan, int *tile) {
    return guarded([&]() -> psp_status {
        if (!p || !plan || !tile) return fail(PSP_EINVAL, "NULL argument");
        shape_to(p->shape, plan, tile);
        return PSP_OK;
    });
}

psp_status psp_tuning_set(int n, psp_dtype dtype, const int *plan, const int *tile) {
    return guarded([&]() -> psp_status {
        if (dtype != PSP_F64 && dtype != PSP_F32) return fail(PSP_EINVAL, "unknown dtype %d", (int)dtype);
        if (n < 4 || n > 384 || (n & 1) || !supported_length(2 * n)) return fail(PSP_EUNSUPPORTED, "unsupported n = %d", n);
        Shape s;
        psp_status rs = shape_from(n, plan, tile, &s);
        if (rs != PSP_OK) return rs;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[{n, dtype == PSP_F32}] = s;
        return PSP_OK;
    });
}

psp_status psp_tuning_get(int n, psp_dtype dtype, int *plan, int *tile) {
    return guarded([&]() -> psp_status {
        if (!plan || !tile) return fail(PSP_EINVAL, "NULL argument");
        if (dtype != PSP_F64 && dtype != PSP_F32) return fail(PSP_EINVAL, "unknown dtype %d", (int)dtype);
        shape_to(tuned_shape(n, dtype == PSP_F32), plan, tile);
        return PSP_OK;
    });
}

psp_status psp_autotune(psp_plan *p, int reps, void *stream, int *best_plan, int *best_tile, float *best_ms,
                        float *cand_ms) {
    return guarded([&]() -> psp_status {
        if (!p) return fail(PSP_EINVAL, "plan is NULL");
        if (reps < 1 || reps > 1000) return fail(PSP_EINVAL, "reps must be in [1, 1000] (got %d)", reps);
        if (!p->precomputed) return fail(PSP_ESTATE, "autotune before psp_kernel_precompute");
        if (p->grid) return fail(PSP_EUNSUPPORTED, "autotune a cube of each axis's size instead");
        {
            std::lock_guard<std::mutex> lk(p->mu);
            if (p->prof_cap > 0) return fail(PSP_ESTATE, "autotune while profiling");
        }
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
            return fail(PSP_EINVAL, "plan was precomputed on device %d, current is %d", p->device, dev);
        hipStream_t st = (hipStream_t)stream;
        Workspace *w = nullptr;
        psp_status rs = plan_workspace(p, st, &w);
        if (rs != PSP_OK) return rs;
        const int n = p->n;
        const bool f32 = p->dtype == PSP_F32;
        const size_t bytes = (size_t)n * n * n * (f32 ? 4 : 8);
        void *rho = nullptr, *rho_b = nullptr, *u = nullptr;
        if (hipMalloc(&rho, bytes) != hipSuccess || hipMalloc(&rho_b, bytes) != hipSuccess ||
            hipMalloc(&u, bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (rho) (void)hipFree(rho);
            if (rho_b) (void)hipFree(rho_b);
            return fail(PSP_ENOMEM, "autotune buffers of %zu bytes failed", 3 * bytes);
        }
        const int nev = solve_launches(n, f32, p->chunk_tiles, p->i1_group) + 1;
        std::vector<hipEvent_t> ev(nev, nullptr);
        std::vector<int> ev_pass(nev, -1);
        std::vector<std::vector<std::pair<int, int>>> cand(kPasses);
        size_t rounds = 0;
        for (int i = 0; i < kPasses; ++i) {
            cand[i] = candidates(n, i);
            rounds = std::max(rounds, cand[i].size());
        }
        // every timing of every candidate; the pick uses the median
        std::vector<std::vector<std::vector<float>>> samples(kPasses);
        for (int i = 0; i < kPasses; ++i) samples[i].resize(cand[i].size());
        psp_status out = PSP_OK;
        const size_t count = (size_t)n * n * n;
        if (f32) {
            hipLaunchKernelGGL(k_fill_hash<float>, dim3(1024), dim3(256), 0, st, (float *)rho, count);
            hipLaunchKernelGGL(k_fill_bump<float>, dim3(1024), dim3(256), 0, st, (float *)rho_b, n);
        } else {
            hipLaunchKernelGGL(k_fill_hash<double>, dim3(1024), dim3(256), 0, st, (double *)rho, count);
            hipLaunchKernelGGL(k_fill_bump<double>, dim3(1024), dim3(256), 0, st, (double *)rho_b, n);
        }
        hipError_t e = hipGetLastError();
        // timing only: no system-scope cache writeback at every record
        for (int k = 0; k < nev && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ev[k], hipEventDisableSystemFence);
        if (e != hipSuccess) out = hip_fail(e, "autotune set-up");
        // round r runs candidate r mod (count) of every pass at once: each pass
        // is timed by its own events, so one round measures five candidates;
        // every round runs on both inputs, and a candidate's samples from
        // both go into its median
        for (size_t r = 0; r < 2 * rounds && out == PSP_OK; ++r) {
            Shape s;
            for (int i = 0; i < kPasses; ++i) {
                const auto &c = cand[i][(r / 2) % cand[i].size()];
                s.plan[i] = c.first;
                s.tile[i] = c.second;
            }
            SolveArgs a = solve_args(p, *w, (r & 1) ? rho_b : rho, u);
            a.shape = s;
            if ((e = launch_solve(a, st)) != hipSuccess) {   // warm-up
                out = hip_fail(e, "autotune launch");
                break;
            }
            a.ev = ev.data();
            a.ev_pass = ev_pass.data();
            a.nev = nev;
            for (int rep = 0; rep < reps && out == PSP_OK; ++rep) {
                if ((e = launch_solve(a, st)) != hipSuccess || (e = hipEventSynchronize(ev[nev - 1])) != hipSuccess) {
                    out = hip_fail(e, "autotune solve");
                    break;
                }
                float pass_ms[kPasses] = {0, 0, 0, 0, 0};
                for (int k = 0; k + 1 < nev; ++k) {
                    float ms = 0;
                    if ((e = hipEventElapsedTime(&ms, ev[k], ev[k + 1])) != hipSuccess) {
                        out = hip_fail(e, "autotune timing");
                        break;
                    }
                    if (ev_pass[k] >= 0 && ev_pass[k] < kPasses) pass_ms[ev_pass[k]] += ms;
                }
                for (int i = 0; i < kPasses; ++i) samples[i][(r / 2) % cand[i].size()].push_back(pass_ms[i]);
            }
        }
        if (out == PSP_OK && (e = hipStreamSynchronize(st)) != hipSuccess) out = hip_fail(e, "autotune");
        // per-pass medians; per pass the fastest candidate unless the default
        // (candidate 0) is within 1%
        std::vector<std::vector<float>> best(kPasses);
        for (int i = 0; i < kPasses; ++i)
            for (auto &v : samples[i]) {
                std::sort(v.begin(), v.end());
                best[i].push_back(v.empty() ? FLT_MAX : v[v.size() / 2]);
            }
        std::vector<size_t> pick(kPasses, 0);
        for (int i = 0; i < kPasses; ++i)
            for (size_t c = 1; c < cand[i].size(); ++c)
                if (best[i][c] < 0.99f * best[i][0] && best[i][c] < best[i][pick[i]]) pick[i] = c;
        auto shape_of = [&](const std::vector<size_t> &pk) {
            Shape s;
            for (int i = 0; i < kPasses; ++i) {
                s.plan[i] = cand[i][pk[i]].first;
                s.tile[i] = cand[i][pk[i]].second;
            }
            return s;
        };
        // Whole-solve refinement.  A pass's launch changes the cache state
        // the next pass starts from (dirty lines, what stays in L2), which
        // per-pass medians over mixed neighbours do not see: a cache policy
        // can slow its own pass and speed up the next one by more.  For each
        // pass in turn, its kRefine fastest candidates and the other cache
        // policies of its current pick are timed as whole solves inside the
        // current pick (reps solves per input, the sum of the two inputs'
        // medians), and a candidate replaces the pick when it is faster by
        // more than 0.2%.
        constexpr size_t kRefine = 4;
        auto whole = [&](const Shape &sh, float *score) -> psp_status {
            *score = 0;
            for (int in = 0; in < 2; ++in) {
                SolveArgs a = solve_args(p, *w, in ? rho_b : rho, u);
                a.shape = sh;
                if ((e = launch_solve(a, st)) != hipSuccess) return hip_fail(e, "autotune launch");   // warm-up
                a.ev = ev.data();
                a.ev_pass = ev_pass.data();
                a.nev = nev;
                std::vector<float> t;
                for (int rep = 0; rep < reps; ++rep) {
                    float ms = 0;
                    if ((e = launch_solve(a, st)) != hipSuccess || (e = hipEventSynchronize(ev[nev - 1])) != hipSuccess ||
                        (e = hipEventElapsedTime(&ms, ev[0], ev[nev - 1])) != hipSuccess)
                        return hip_fail(e, "autotune solve");
                    t.push_back(ms);
                }
                std::sort(t.begin(), t.end());
                *score += t[t.size() / 2];
            }
            return PSP_OK;
        };
        float cur = 0;
        if (out == PSP_OK) out = whole(shape_of(pick), &cur);
        for (int i = 0; i < kPasses && out == PSP_OK; ++i) {
            std::vector<size_t> order(cand[i].size());
            for (size_t c = 0; c < order.size(); ++c) order[c] = c;
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return best[i][a] < best[i][b]; });
            order.resize(std::min(kRefine, order.size()));
            // the same plan and tile shape under the pass's other cache policies
            const int stride = (i == 0 || i == 4) ? 4 : 7;
            const int pl = cand[i][pick[i]].first, shape_t = cand[i][pick[i]].second % stride;
            for (size_t c = 0; c < cand[i].size(); ++c)
                if (cand[i][c].first == pl && cand[i][c].second % stride == shape_t &&
                    std::find(order.begin(), order.end(), c) == order.end())
                    order.push_back(c);
            const std::vector<size_t> base = pick;
            for (size_t k = 0; k < order.size() && out == PSP_OK; ++k) {
                if (order[k] == base[i] || order[k] == pick[i]) continue;
                std::vector<size_t> trial = pick;
                trial[i] = order[k];
                float score = 0;
                out = whole(shape_of(trial), &score);
                if (out == PSP_OK && score < 0.998f * cur) {
                    pick = trial;
                    cur = score;
                }
            }
        }
        if (out == PSP_OK && (e = hipStreamSynchronize(st)) != hipSuccess) out = hip_fail(e, "autotune");
        for (auto x : ev)
            if (x) (void)hipEventDestroy(x);
        (void)hipFree(rho);
        (void)hipFree(rho_b);
        (void)hipFree(u);
        if (out != PSP_OK) return out;
        const Shape chosen = shape_of(pick);
        if (best_ms)
            for (int i = 0; i < kPasses; ++i) best_ms[i] = best[i][pick[i]];
        {
            std::lock_guard<std::mutex> lk(p->mu);
            p->shape = chosen;
        }
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[{n, f32}] = chosen;
        }
        shape_to(chosen, best_plan, best_tile);
        if (cand_ms) {
            constexpr int stride = kMaxPlans * kMaxTiles;
            for (int i = 0; i < kPasses * stride; ++i) cand_ms[i] = -1.0f;
            for (int i = 0; i < kPasses; ++i)
                for (size_t c = 0; c < cand[i].size(); ++c)
                    cand_ms[i * stride + cand[i][c].first * kMaxTiles + cand[i][c].second] = best[i][c];
        }
        return PSP_OK;
    });
}

}  // extern "C"
