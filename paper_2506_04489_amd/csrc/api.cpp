// api.cpp - libpsp's C ABI: plans, precompute, solves, test hooks, errors.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <tuple>

#include "host_common.hpp"

namespace psp {

static thread_local std::string g_last_error;

psp_status fail(psp_status e, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    try {
        g_last_error = buf;
    } catch (...) {   // out of host memory: keep the previous detail
    }
    return e;
}

psp_status hip_fail(hipError_t err, const char *what) {
    return fail(PSP_EHIP, "%s: %s", what, hipGetErrorString(err));
}

#define PSP_HIP(call, what)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

DevSpectrum::~DevSpectrum() {
    if (mult) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != device) (void)hipSetDevice(device);
        (void)hipFree(mult);
        if (cur != device && cur >= 0) (void)hipSetDevice(cur);
    }
}

// ---------------------------------------------------------------- caches
static std::mutex g_cache_mu;
// device, n[3], h[3], R, eps, delta
using SpecKey = std::tuple<int, int, int, int, double, double, double, int, double, double>;
static std::map<SpecKey, std::weak_ptr<DevSpectrum>> g_spec_cache;
static std::map<std::pair<int, int>, Twiddles> g_tw_cache;            // (device, N)

psp_status get_twiddles(int device, int N, const Twiddles **out) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto key = std::make_pair(device, N);
    auto it = g_tw_cache.find(key);
    if (it != g_tw_cache.end()) {
        *out = &it->second;
        return PSP_OK;
    }
    std::vector<double> w(2 * (size_t)N);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int m = 0; m < N; ++m) {
        // exp(-2 pi i m / N), long double evaluation rounded once
        const long double ang = two_pi * (long double)m / (long double)N;
        const double c = (double)cosl(ang), s = (double)-sinl(ang);
        w[2 * m] = c;
        w[2 * m + 1] = s;
    }
    Twiddles t;
    PSP_HIP(hipMalloc(&t.w64, w.size() * 8), "hipMalloc(twiddles)");
    PSP_HIP(hipMemcpy(t.w64, w.data(), w.size() * 8, hipMemcpyHostToDevice), "hipMemcpy(twiddles)");
    auto res = g_tw_cache.emplace(key, t);
    *out = &res.first->second;
    return PSP_OK;
}

psp_status check_create(int n, double h, int R, double eps, double delta) {
    if (!(h > 0.0) || !std::isfinite(h)) return fail(PSP_EINVAL, "h must be positive and finite (got %g)", h);
    if (R < 1 || R > 2048) return fail(PSP_EINVAL, "R must be in [1, 2048] (got %d)", R);
    if (!(eps > 0.0) || !(delta > eps) || !std::isfinite(delta))
        return fail(PSP_EINVAL, "need 0 < eps < delta finite (got %g, %g)", eps, delta);
    if (n < 4 || n > 384 || (n & 1)) return fail(PSP_EUNSUPPORTED, "n must be even and in [4, 384] (got %d)", n);
    if (!supported_length(2 * n))
        return fail(PSP_EUNSUPPORTED, "2n = %d is not of the form 2^a 3^b (n = %d)", 2 * n, n);
    return PSP_OK;
}

static std::atomic<bool> g_guards{false};
bool guards_enabled() { return g_guards.load(); }

// one device buffer of `bytes`, inside pattern-filled guard bands when asked
static hipError_t guarded_malloc(size_t bytes, bool guard, void **base, void **buf) {
    const size_t total = guard ? bytes + 2 * kGuardBytes : bytes;
    hipError_t e = hipMalloc(base, total);
    if (e != hipSuccess) {
        *base = nullptr;
        return e;
    }
    *buf = guard ? (unsigned char *)*base + kGuardBytes : *base;
    if (guard) {
        e = hipMemset(*base, kGuardByte, kGuardBytes);
        if (e == hipSuccess) e = hipMemset((unsigned char *)*buf + bytes, kGuardByte, kGuardBytes);
    }
    return e;
}

psp_status alloc_workspace(int n, bool f32, int chunk_tiles, Workspace *w, int i1_group) {
    const size_t c = f32 ? 8 : 16, P = (size_t)pitch_for(n);
    const size_t plane = a_plane(n, n, chunk_pitch(n, f32, chunk_tiles), (int)c);
    const size_t xs = (size_t)x_slabs(n, f32, chunk_tiles, i1_group);
    const bool guard = guards_enabled();
    w->bytes = workspace_bytes(n, f32, chunk_tiles, i1_group);
    w->X = w->A = w->X_base = w->A_base = nullptr;
    w->X_bytes = c * P * xs * n;
    w->A_bytes = c * plane * n;
    if (guarded_malloc(w->X_bytes, guard, &w->X_base, &w->X) != hipSuccess) {
        (void)hipGetLastError();
        free_workspace(w);
        return fail(PSP_ENOMEM, "workspace allocation of %zu bytes failed", w->bytes);
    }
    if (guarded_malloc(w->A_bytes, guard, &w->A_base, &w->A) != hipSuccess) {
        (void)hipGetLastError();
        free_workspace(w);
        return fail(PSP_ENOMEM, "workspace allocation of %zu bytes failed", w->bytes);
    }
    return PSP_OK;
}

psp_status alloc_workspace_dims(const Dims &d, bool f32, Workspace *w) {
    const size_t c = f32 ? 8 : 16, P = (size_t)pitch_for(d.n3);
    const size_t plane = a_plane(d.n1, d.n2, chunk_pitch(d.n3, f32, 0), (int)c);
    const bool guard = guards_enabled();
    w->bytes = workspace_bytes_dims(d, f32);
    w->X = w->A = w->X_base = w->A_base = nullptr;
    w->X_bytes = c * P * (size_t)d.n1 * d.n2;
    w->A_bytes = c * plane * (size_t)d.n1;
    if (guarded_malloc(w->X_bytes, guard, &w->X_base, &w->X) != hipSuccess ||
        guarded_malloc(w->A_bytes, guard, &w->A_base, &w->A) != hipSuccess) {
        (void)hipGetLastError();
        free_workspace(w);
        return fail(PSP_ENOMEM, "workspace allocation of %zu bytes failed", w->bytes);
    }
    return PSP_OK;
}

void free_workspace(Workspace *w) {
    if (w->X_base) (void)hipFree(w->X_base);
    if (w->A_base) (void)hipFree(w->A_base);
    w->X = w->A = w->X_base = w->A_base = nullptr;
}

psp_status check_guards(const Workspace &w, bool *intact) {
    *intact = true;
    std::vector<unsigned char> band(kGuardBytes);
    const std::pair<void *, void *> bufs[2] = {{w.X_base, w.X}, {w.A_base, w.A}};
    const size_t sizes[2] = {w.X_bytes, w.A_bytes};
    for (int i = 0; i < 2; ++i) {
        if (!bufs[i].first || bufs[i].first == bufs[i].second) continue;   // not guarded
        const unsigned char *ends[2] = {(const unsigned char *)bufs[i].first,
                                        (const unsigned char *)bufs[i].second + sizes[i]};
        for (const unsigned char *e : ends) {
            PSP_HIP(hipMemcpy(band.data(), e, kGuardBytes, hipMemcpyDeviceToHost), "hipMemcpy(guard)");
            for (unsigned char b : band)
                if (b != kGuardByte) {
                    *intact = false;
                    return PSP_OK;
                }
        }
    }
    return PSP_OK;
}

psp_status plan_workspace(const psp_plan *p, hipStream_t st, Workspace **out) {
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->ws.find(st);
    if (it != p->ws.end()) {
        *out = &it->second;
        return PSP_OK;
    }
    Workspace w;
    psp_status rs = p->grid ? alloc_workspace_dims(Dims{p->ns[0], p->ns[1], p->ns[2]}, p->dtype == PSP_F32, &w)
                            : alloc_workspace(p->n, p->dtype == PSP_F32, p->chunk_tiles, &w, p->i1_group);
    if (rs != PSP_OK) return rs;
    auto res = p->ws.emplace(st, w);
    *out = &res.first->second;
    return PSP_OK;
}

SolveArgs solve_args(const psp_plan *p, const Workspace &w, const void *rho, void *u) {
    SolveArgs a;
    a.n = p->n;
    a.P = pitch_for(p->n);
    a.f32 = p->dtype == PSP_F32;
    a.rho = rho;
    a.u = u;
    a.X = w.X;
    a.A = w.A;
    a.chunk_tiles = p->chunk_tiles;
    a.i1_group = p->i1_group;
    a.shape = p->shape;
    a.mult = p->spec->mult;
    a.tw64 = p->tw->w64;
    if (p->grid) {
        a.P = pitch_for(p->ns[2]);
        for (int i = 0; i < 3; ++i) {
            a.ns[i] = p->ns[i];
            a.tw_axis[i] = p->tws[i]->w64;
        }
    }
    return a;
}

// S1 on the device, once per distinct axis period: one allocation holding,
// per distinct period, J0 and J2 (R x (n+1) each), then the Gaussian-sum
// weights (R), the quadrature layouts (R jobs per period) and the
// trigonometric table; the tables are filled on `st`.  tb receives the table
// pointers of axes 1..3 (shared where the periods coincide) and *omega the
// device weights.  The caller frees *buf after the stream has run, and keeps
// `hold` (the host copies being uploaded) alive until then.
struct TableUpload {
    std::vector<std::vector<TabJob>> jobs;
    std::vector<TabTrig> trig;
};
static psp_status device_tables(const psp_plan *p, hipStream_t st, TableUpload &hold, double **buf, SpecTables *tb,
                                const double **omega) {
    std::vector<std::pair<int, double>> axes;   // distinct (points, period)
    int axis_of[3];
    for (int a = 0; a < 3; ++a) {
        const std::pair<int, double> key{p->ns[a], p->Ls[a]};
        auto it = std::find(axes.begin(), axes.end(), key);
        axis_of[a] = (int)(it - axes.begin());
        if (it == axes.end()) axes.push_back(key);
    }
    const int nd = (int)axes.size();
    std::vector<size_t> off(nd + 1, 0);           // doubles before distinct axis i
    for (int i = 0; i < nd; ++i) off[i + 1] = off[i] + 2 * (size_t)p->R * (axes[i].first + 1);
    hold.trig = table_trig();
    hold.jobs.clear();
    for (int i = 0; i < nd; ++i) hold.jobs.push_back(table_jobs(p->alpha, axes[i].first, axes[i].second));
    double *d = nullptr;
    PSP_HIP(hipMalloc(&d, sizeof(double) * (off[nd] + p->R) + sizeof(TabJob) * p->R * nd +
                              sizeof(TabTrig) * hold.trig.size()),
            "hipMalloc(tables)");
    *buf = d;
    double *dw = d + off[nd];
    TabJob *dj = reinterpret_cast<TabJob *>(dw + p->R);
    TabTrig *dt = reinterpret_cast<TabTrig *>(dj + (size_t)p->R * nd);
    hipError_t e = hipMemcpyAsync(dw, p->omega.data(), sizeof(double) * p->R, hipMemcpyHostToDevice, st);
    for (int i = 0; i < nd && e == hipSuccess; ++i) {
        const size_t tn = (size_t)p->R * (axes[i].first + 1);
        e = launch_tables(hold.jobs[i], hold.trig, axes[i].first, axes[i].second, d + off[i], d + off[i] + tn,
                          dj + (size_t)p->R * i, dt, st);
    }
    if (e != hipSuccess) return hip_fail(e, "1D tables");
    for (int a = 0; a < 3; ++a) {
        const int i = axis_of[a];
        tb->J0[a] = d + off[i];
        tb->J2[a] = d + off[i] + (size_t)p->R * (axes[i].first + 1);
        tb->n[a] = p->ns[a];
    }
    *omega = dw;
    return PSP_OK;
}

static psp_status current_device_of(const psp_plan *p) {
    int dev = -1;
    PSP_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) return fail(PSP_EINVAL, "plan was precomputed on device %d, current is %d", p->device, dev);
    return PSP_OK;
}

}  // namespace psp

using namespace psp;

extern "C" {

const char *psp_strerror(psp_status e) {
    switch (e) {
        case PSP_OK: return "success";
        case PSP_EINVAL: return "invalid argument";
        case PSP_ENOMEM: return "out of memory";
        case PSP_EUNSUPPORTED: return "unsupported size";
        case PSP_ESTATE: return "invalid call order";
        case PSP_EHIP: return "HIP runtime error";
        case PSP_EBUSY: return "busy";
        case PSP_ECANCELED: return "canceled";
    }
    return "unknown status";
}

const char *psp_last_error(void) { return g_last_error.c_str(); }

// a plan for ns[p] points and spacing hs[p] along axis p, explicit cutoff
static psp_status create_plan(const int *ns, const double *hs, int R, psp_dtype dtype, double eps, double delta,
                              psp_plan **out) {
    if (!out) return fail(PSP_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != PSP_F64 && dtype != PSP_F32) return fail(PSP_EINVAL, "unknown dtype %d", (int)dtype);
    for (int a = 0; a < 3; ++a) {
        psp_status st = check_create(ns[a], hs[a], R, eps, delta);
        if (st != PSP_OK) return st;
    }
    psp_plan *p = new (std::nothrow) psp_plan;
    if (!p) return fail(PSP_ENOMEM, "host allocation failed");
    const int n = ns[0];
    p->n = n;
    p->grid = !(ns[0] == ns[1] && ns[1] == ns[2]);
    for (int a = 0; a < 3; ++a) {
        p->ns[a] = ns[a];
        p->hs[a] = hs[a];
        p->Ls[a] = 2.0 * ns[a] * hs[a];
    }
    p->h = hs[0];
    p->L = p->Ls[0];
    p->R = R;
    p->dtype = dtype;
    p->eps = eps;
    p->delta = delta;
    p->chunk_tiles = 0;   // one chunk: fastest for a single solve
    p->shape = tuned_shape(n, dtype == PSP_F32);
    if (p->grid) {
        // each pass takes the tuned shape of its own axis's length
        static const int axis_of_pass[kPasses] = {2, 1, 0, 1, 2};
        for (int q = 0; q < kPasses; ++q) {
            const Shape s = tuned_shape(ns[axis_of_pass[q]], dtype == PSP_F32);
            p->shape.plan[q] = s.plan[q];
            p->shape.tile[q] = s.tile[q];
        }
    }
    gs_fit(R, eps, delta, p->omega, p->alpha);
    *out = p;
    return PSP_OK;
}

psp_status psp_plan_create_ex(int n, double h, int R, psp_dtype dtype, double eps, double delta, psp_plan **out) {
    return guarded([&]() -> psp_status {
        const int ns[3] = {n, n, n};
        const double hs[3] = {h, h, h};
        return create_plan(ns, hs, R, dtype, eps, delta, out);
    });
}

psp_status psp_plan_create_grid(const int *n, const double *h, int R, psp_dtype dtype, double eps, double delta,
                                psp_plan **out) {
    return guarded([&]() -> psp_status {
        if (!out) return fail(PSP_EINVAL, "out is NULL");
        *out = nullptr;
        if (!n || !h) return fail(PSP_EINVAL, "n or h is NULL");
        if (eps <= 0.0 && delta <= 0.0) {
            // eps = 1e-4 max_p L_p/2 and delta = |(L_1, L_2, L_3)|/2, the corner
            // of the kernel's truncation box (L_p = 2 n_p h_p)
            double mx = 0.0, sq = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double half = (double)n[a] * h[a];
                mx = std::max(mx, half);
                sq += half * half;
            }
            eps = 1e-4 * mx;
            delta = std::sqrt(sq);
        }
        return create_plan(n, h, R, dtype, eps, delta, out);
    });
}

psp_status psp_plan_create_box(int n, const double *h, int R, psp_dtype dtype, double eps, double delta,
                               psp_plan **out) {
    return guarded([&]() -> psp_status {
        const int ns[3] = {n, n, n};
        return psp_plan_create_grid(ns, h, R, dtype, eps, delta, out);
    });
}

psp_status psp_plan_create(int n, double h, int R, psp_dtype dtype, psp_plan **out) {
    return guarded([&]() -> psp_status {
        // eps = 1e-4 L/2 and delta = sqrt(3) L/2 with L = 2 n h (the default cutoff
        // in units where L = 2, and the corner of the kernel's truncation box)
        const double half = (double)n * h;
        return psp_plan_create_ex(n, h, R, dtype, 1e-4 * half, std::sqrt(3.0) * half, out);
    });
}

static void profile_clear(psp_plan *p) {
    for (auto e : p->prof_ev) (void)hipEventDestroy(e);
    p->prof_ev.clear();
    p->prof_pass.clear();
    p->prof_cap = p->prof_used = 0;
}

void psp_plan_destroy(psp_plan *p) {
    try {
        if (!p) return;
        profile_clear(p);
        for (auto &kv : p->ws) free_workspace(&kv.second);
        delete p;
    } catch (...) {
    }
}

psp_status psp_plan_get_gs(const psp_plan *p, double *omega, double *alpha) {
    return guarded([&]() -> psp_status {
        if (!p || !omega || !alpha) return fail(PSP_EINVAL, "NULL argument");
        std::memcpy(omega, p->omega.data(), sizeof(double) * p->R);
        std::memcpy(alpha, p->alpha.data(), sizeof(double) * p->R);
        return PSP_OK;
    });
}

psp_status psp_plan_get_tables(psp_plan *p, double *J0, double *J2) {
    return guarded([&]() -> psp_status {
        if (!p || !J0 || !J2) return fail(PSP_EINVAL, "NULL argument");
        if (p->precomputed) {
            psp_status s = current_device_of(p);
            if (s != PSP_OK) return s;
        }
        TableUpload hold;
        SpecTables tabs;
        const double *dw = nullptr;
        double *d = nullptr;
        psp_status rs = device_tables(p, nullptr, hold, &d, &tabs, &dw);
        const size_t tb = sizeof(double) * (size_t)p->R * (p->n + 1);
        hipError_t e = hipSuccess;
        if (rs == PSP_OK && (e = hipMemcpy(J0, tabs.J0[0], tb, hipMemcpyDeviceToHost)) == hipSuccess)
            e = hipMemcpy(J2, tabs.J2[0], tb, hipMemcpyDeviceToHost);
        if (d) (void)hipFree(d);
        if (rs != PSP_OK) return rs;
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(tables)");
        return PSP_OK;
    });
}

psp_status psp_plan_workspace_bytes(const psp_plan *p, size_t *bytes) {
    return guarded([&]() -> psp_status {
        if (!p || !bytes) return fail(PSP_EINVAL, "NULL argument");
        *bytes = p->grid ? workspace_bytes_dims(Dims{p->ns[0], p->ns[1], p->ns[2]}, p->dtype == PSP_F32)
                         : workspace_bytes(p->n, p->dtype == PSP_F32, p->chunk_tiles, p->i1_group);
        return PSP_OK;
    });
}

psp_status psp_plan_spectrum_bytes(const psp_plan *p, size_t *bytes) {
    return guarded([&]() -> psp_status {
        if (!p || !bytes) return fail(PSP_EINVAL, "NULL argument");
        *bytes = p->grid ? spectrum_bytes_dims(Dims{p->ns[0], p->ns[1], p->ns[2]}) : spectrum_bytes(p->n);
        return PSP_OK;
    });
}

psp_status psp_kernel_precompute(psp_plan *p, void *stream) {
    return guarded([&]() -> psp_status {
        if (!p) return fail(PSP_EINVAL, "plan is NULL");
        hipStream_t st = (hipStream_t)stream;
        if (p->precomputed) return current_device_of(p);
        int dev = -1;
        PSP_HIP(hipGetDevice(&dev), "hipGetDevice");
        for (int a = 0; a < 3; ++a) {
            psp_status rs = get_twiddles(dev, 2 * p->ns[a], &p->tws[a]);
            if (rs != PSP_OK) return rs;
        }
        p->tw = p->tws[0];
        const SpecKey key{dev, p->ns[0], p->ns[1], p->ns[2], p->hs[0], p->hs[1], p->hs[2], p->R, p->eps, p->delta};
        std::shared_ptr<DevSpectrum> spec;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_spec_cache.find(key);
            if (it != g_spec_cache.end()) spec = it->second.lock();
        }
        if (!spec) {
            const int R = p->R, P = pitch_for(p->ns[2]);
            spec = std::make_shared<DevSpectrum>();
            spec->device = dev;
            spec->bytes = spectrum_bytes_dims(Dims{p->ns[0], p->ns[1], p->ns[2]});
            hipError_t e = hipMalloc(&spec->mult, spec->bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                spec->mult = nullptr;
                return fail(PSP_ENOMEM, "spectrum allocation of %zu bytes failed", spec->bytes);
            }
            TableUpload hold;
            SpecTables tabs;
            const double *dW = nullptr;
            double *dJ = nullptr;
            psp_status out = device_tables(p, st, hold, &dJ, &tabs, &dW);
            do {
                if (out != PSP_OK) break;
                hipError_t ee;
                if ((ee = hipMemsetAsync(spec->mult, 0, spec->bytes, st)) != hipSuccess) {
                    out = hip_fail(ee, "precompute upload");
                    break;
                }
                const double pi = 3.14159265358979323846;
                SpecScale sc;
                for (int a = 0; a < 3; ++a) sc.w[a] = (2.0 * pi / p->Ls[a]) * (2.0 * pi / p->Ls[a]);
                sc.scale = -1.0 / ((2.0 * p->ns[0]) * (2.0 * p->ns[1]) * (2.0 * p->ns[2]));
                if ((ee = launch_spectrum(tabs, dW, R, P, sc, spec->mult, st)) != hipSuccess) {
                    out = hip_fail(ee, "spectrum kernel launch");
                    break;
                }
                if ((ee = hipStreamSynchronize(st)) != hipSuccess) {
                    out = hip_fail(ee, "spectrum kernel");
                    break;
                }
            } while (0);
            if (dJ) {
                if (out != PSP_OK) (void)hipStreamSynchronize(st);   // nothing may still read it
                (void)hipFree(dJ);
            }
            if (out != PSP_OK) return out;
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_spec_cache[key] = spec;
        }
        p->spec = spec;
        p->device = dev;
        p->precomputed = true;
        return PSP_OK;
    });
}

psp_status psp_plan_get_multiplier(psp_plan *p, double *m_host) {
    return guarded([&]() -> psp_status {
        if (!p || !m_host) return fail(PSP_EINVAL, "NULL argument");
        if (!p->precomputed) return fail(PSP_ESTATE, "multiplier requested before psp_kernel_precompute");
        const Dims d{p->ns[0], p->ns[1], p->ns[2]};
        const int P = pitch_for(d.n3);
        const size_t bytes = spectrum_bytes_dims(d);
        std::vector<double> blk(bytes / 8);
        PSP_HIP(hipMemcpy(blk.data(), p->spec->mult, bytes, hipMemcpyDeviceToHost), "hipMemcpy(mult)");
        const size_t na = (size_t)d.n1 + 1, nb = (size_t)d.n2 + 1, nc = (size_t)d.n3 + 1;
        for (size_t a = 0; a < na; ++a)
            for (size_t b = 0; b < nb; ++b)
                for (size_t c = 0; c < nc; ++c)
                    m_host[(a * nb + b) * nc + c] = blk[((b * (P / 8) + c / 8) * na + a) * 8 + (c & 7)];
        return PSP_OK;
    });
}

psp_status psp_solve(const psp_plan *p, const void *rho_dev, void *u_dev, void *stream) {
    return guarded([&]() -> psp_status {
        if (!p || !rho_dev || !u_dev) return fail(PSP_EINVAL, "NULL argument");
        if (!p->precomputed) return fail(PSP_ESTATE, "psp_solve before psp_kernel_precompute");
        if (rho_dev == u_dev) return fail(PSP_EINVAL, "rho and u must not alias");
        psp_status st = current_device_of(p);
        if (st != PSP_OK) return st;
        Workspace *w = nullptr;
        st = plan_workspace(p, (hipStream_t)stream, &w);
        if (st != PSP_OK) return st;
        SolveArgs a = solve_args(p, *w, rho_dev, u_dev);
        {
            std::lock_guard<std::mutex> lk(p->mu);
            if (p->prof_used < p->prof_cap) {
                a.ev = &p->prof_ev[(size_t)p->prof_nev * p->prof_used];
                a.ev_pass = &p->prof_pass[(size_t)p->prof_nev * p->prof_used];
                a.nev = p->prof_nev;
                p->prof_used++;
            }
        }
        hipError_t e = launch_solve(a, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "solve launch");
        return PSP_OK;
    });
}

psp_status psp_profile_enable(psp_plan *p, int max_solves) {
    return guarded([&]() -> psp_status {
        if (!p || max_solves < 0 || max_solves > 100000) return fail(PSP_EINVAL, "bad profile arguments");
        if (p->grid) return fail(PSP_EUNSUPPORTED, "per-pass profiling needs equal point counts per axis");
        std::lock_guard<std::mutex> lk(p->mu);
        profile_clear(p);
        p->prof_nev = solve_launches(p->n, p->dtype == PSP_F32, p->chunk_tiles, p->i1_group) + 1;
        p->prof_ev.resize((size_t)p->prof_nev * max_solves, nullptr);
        p->prof_pass.assign((size_t)p->prof_nev * max_solves, -1);
        for (auto &e : p->prof_ev) {
            // timing only: no system-scope cache writeback at every record
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
                e = nullptr;
                profile_clear(p);
                return fail(PSP_EHIP, "hipEventCreate failed");
            }
        }
        p->prof_cap = max_solves;
        return PSP_OK;
    });
}

psp_status psp_profile_read(psp_plan *p, int *count, double *pass_ms) {
    return guarded([&]() -> psp_status {
        if (!p || !count || !pass_ms) return fail(PSP_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(p->mu);
        for (int i = 0; i < 6; ++i) pass_ms[i] = 0.0;
        *count = p->prof_used;
        const int nev = p->prof_nev;
        for (int k = 0; k < p->prof_used; ++k) {
            hipEvent_t *ev = &p->prof_ev[(size_t)nev * k];
            const int *pass = &p->prof_pass[(size_t)nev * k];
            PSP_HIP(hipEventSynchronize(ev[nev - 1]), "hipEventSynchronize");
            for (int i = 0; i + 1 < nev; ++i) {
                float ms = 0;
                PSP_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "hipEventElapsedTime");
                if (pass[i] >= 0 && pass[i] < 5) pass_ms[pass[i]] += ms;
            }
            float tot = 0;
            PSP_HIP(hipEventElapsedTime(&tot, ev[0], ev[nev - 1]), "hipEventElapsedTime");
            pass_ms[5] += tot;
        }
        if (p->prof_used > 0)
            for (int i = 0; i < 6; ++i) pass_ms[i] /= p->prof_used;
        profile_clear(p);
        return PSP_OK;
    });
}

psp_status psp_plan_set_tuning(psp_plan *p, int k3_tiles, int i1_group) {
    return guarded([&]() -> psp_status {
        if (!p || k3_tiles < 0 || i1_group < 0) return fail(PSP_EINVAL, "bad tuning arguments");
        if (p->grid && (k3_tiles != 0 || i1_group != 0))
            return fail(PSP_EUNSUPPORTED, "k3 chunks and i1 groups need equal point counts per axis");
        std::lock_guard<std::mutex> lk(p->mu);
        if (p->prof_cap > 0) return fail(PSP_ESTATE, "cannot change the tuning while profiling");
        if (k3_tiles != p->chunk_tiles || i1_group != p->i1_group) {
            // existing workspaces were sized for the old layout
            if (!p->ws.empty()) (void)hipDeviceSynchronize();
            for (auto &kv : p->ws) free_workspace(&kv.second);
            p->ws.clear();
            p->chunk_tiles = k3_tiles;
            p->i1_group = i1_group;
        }
        return PSP_OK;
    });
}

psp_status psp_debug_guards(int enable) {
    return guarded([&]() -> psp_status {
        g_guards.store(enable != 0);
        return PSP_OK;
    });
}

psp_status psp_plan_check_guards(psp_plan *p, int *intact) {
    return guarded([&]() -> psp_status {
        if (!p || !intact) return fail(PSP_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(p->mu);
        PSP_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        bool all = true;
        for (auto &kv : p->ws) {
            bool ok = true;
            psp_status st = check_guards(kv.second, &ok);
            if (st != PSP_OK) return st;
            all = all && ok;
        }
        *intact = all ? 1 : 0;
        return PSP_OK;
    });
}

psp_status psp_solve_padded_debug(const psp_plan *p, const void *rho_dev, void *upad_dev, void *stream) {
    return guarded([&]() -> psp_status {
        if (!p || !rho_dev || !upad_dev) return fail(PSP_EINVAL, "NULL argument");
        if (!p->precomputed) return fail(PSP_ESTATE, "psp_solve_padded_debug before psp_kernel_precompute");
        if (p->grid) return fail(PSP_EUNSUPPORTED, "the uncropped output needs equal point counts per axis");
        // the uncropped passes run over one chunk of all k3 tiles and every i1
        // slab, which a workspace shrunk by psp_plan_set_tuning cannot hold
        if (p->chunk_tiles != 0 || p->i1_group != 0)
            return fail(PSP_EUNSUPPORTED, "the uncropped output needs the default tuning (no k3 chunks, no i1 groups)");
        psp_status st = current_device_of(p);
        if (st != PSP_OK) return st;
        hipStream_t s = (hipStream_t)stream;
        Workspace *w = nullptr;
        st = plan_workspace(p, s, &w);
        if (st != PSP_OK) return st;
        SolveArgs a = solve_args(p, *w, rho_dev, upad_dev);
        a.full = true;
        const size_t c = a.f32 ? 8 : 16, N = 2 * (size_t)p->n;
        const size_t big = c * N * N * (size_t)a.P;
        PSP_HIP(hipMalloc(&a.A2, big), "hipMalloc(debug)");
        if (hipMalloc(&a.Y2, big) != hipSuccess) {
            (void)hipFree(a.A2);
            return fail(PSP_ENOMEM, "debug allocation failed");
        }
        hipError_t e = launch_solve(a, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(a.A2);
        (void)hipFree(a.Y2);
        if (e != hipSuccess) return hip_fail(e, "padded debug solve");
        return PSP_OK;
    });
}

}  // extern "C"
