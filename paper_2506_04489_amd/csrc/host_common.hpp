// host_common.hpp - shared internal declarations of libpsp's host code.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <map>
#include <new>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/psp.h"
#include "kernels.h"
#include "tables.hpp"

namespace psp {

// thread-local error detail; returns e for convenience
psp_status fail(psp_status e, const char *fmt, ...);
psp_status hip_fail(hipError_t err, const char *what);

// Runs an entry point's body so that no C++ exception crosses the C ABI: a
// failed host allocation becomes PSP_ENOMEM, anything else PSP_EHIP.
template <typename F> psp_status guarded(F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(PSP_ENOMEM, "host memory allocation failed");
    } catch (const std::exception &e) {
        return fail(PSP_EHIP, "internal error: %s", e.what());
    } catch (...) {
        return fail(PSP_EHIP, "internal error");
    }
}

// ---- S0: Gaussian-sum weights and exponents (sinc quadrature) -------------
void gs_fit(int R, double eps, double delta, std::vector<double> &omega, std::vector<double> &alpha);

// ---- S1: 1D integrals of the separable kernel transform (on the device) ---
// J0[s*(n+1)+k] = int_{-L/2}^{L/2} exp(-a_s y^2) cos(2 pi k y / L) dy, J2 with y^2.
// table_jobs: the per-Gaussian quadrature layout; launch_tables copies it and
// the trigonometric table to jobs_dev (R entries) and trig_dev (`jobs` and
// `trig` must stay alive until the stream has run) and fills J0, J2
// (R x (n+1) device doubles each).
std::vector<TabJob> table_jobs(const std::vector<double> &alpha, int n, double L);
std::vector<TabTrig> table_trig();   // TAB_TRIG / 2 + 1 entries
TabRule table_rule();
hipError_t launch_tables(const std::vector<TabJob> &jobs, const std::vector<TabTrig> &trig, int n, double L,
                         double *J0, double *J2, TabJob *jobs_dev, TabTrig *trig_dev, hipStream_t st);

// ---- device resources ------------------------------------------------------
struct DevSpectrum {            // the multiplier octant, shared between plans
    int device = -1;
    double *mult = nullptr;     // blocked layout, (n+1)*P*(n+1) doubles
    size_t bytes = 0;
    ~DevSpectrum();
};

struct Twiddles {               // per (device, N), process lifetime
    void *w64 = nullptr;        // double2[N]: W^m = exp(-2 pi i m / N), m < N
};
psp_status get_twiddles(int device, int N, const Twiddles **out);

struct Workspace {
    void *X = nullptr;
    void *A = nullptr;
    size_t bytes = 0;
    // debug guards (psp_debug_guards): X and A sit kGuardBytes into their
    // allocations, with pattern-filled bands of that size on both sides
    void *X_base = nullptr, *A_base = nullptr;
    size_t X_bytes = 0, A_bytes = 0;
};
constexpr size_t kGuardBytes = 64 * 1024;
constexpr unsigned char kGuardByte = 0xA5;
// whether workspaces allocated from now on carry guards
bool guards_enabled();
// the guard bands of w are intact (reads them back; synchronous)
psp_status check_guards(const Workspace &w, bool *intact);

inline int pitch_for(int n) { return ((n + 1 + 15) / 16) * 16; }
// k3 columns of the H2-H4 chunk buffer for a chunk of `chunk_tiles` tiles
inline int chunk_pitch(int n, bool f32, int chunk_tiles) {
    const int W = strided_width(f32), ntile = (n + 1 + W - 1) / W;
    const int ct = chunk_tiles > 0 && chunk_tiles < ntile ? chunk_tiles : ntile;
    return ct * W;
}
// i1 slabs the X buffer holds: one group when i1 grouping applies (one chunk)
inline int x_slabs(int n, bool f32, int chunk_tiles, int i1_group) {
    const int W = strided_width(f32), ntile = (n + 1 + W - 1) / W;
    const bool one_chunk = chunk_tiles <= 0 || chunk_tiles >= ntile;
    return (one_chunk && i1_group > 0 && i1_group < n) ? i1_group : n;
}
inline size_t workspace_bytes(int n, bool f32, int chunk_tiles, int i1_group = 0) {
    const size_t c = f32 ? 8 : 16;
    const size_t P = (size_t)pitch_for(n);
    const size_t plane = a_plane(n, n, chunk_pitch(n, f32, chunk_tiles), (int)c);
    return c * (P * (size_t)x_slabs(n, f32, chunk_tiles, i1_group) * n + plane * (size_t)n);
}
psp_status alloc_workspace(int n, bool f32, int chunk_tiles, Workspace *w, int i1_group = 0);
// unequal point counts per axis: X holds n1 x n2 rows of pitch P(n3), A the
// one chunk: n1 planes of 2 n2 rows of round_up(n3 + 1, tile) columns
inline size_t workspace_bytes_dims(const Dims &d, bool f32) {
    const size_t c = f32 ? 8 : 16;
    const size_t P = (size_t)pitch_for(d.n3);
    const size_t plane = a_plane(d.n1, d.n2, chunk_pitch(d.n3, f32, 0), (int)c);
    return c * (P * (size_t)d.n1 * d.n2 + plane * (size_t)d.n1);
}
psp_status alloc_workspace_dims(const Dims &d, bool f32, Workspace *w);

// ---- batches: the device image of a batch -----------------------------------
struct BatchMember {
    Job job;                      // pointers; workspace of one chunk holding all tiles
    int n = 0;
    Shape shape;
    const void *tw64 = nullptr;  // twiddles of length 2n
};
struct BatchImage {
    std::vector<int> persist;     // members on the persistent path (2n <= PB_MAX_N), in table order
    std::vector<int> grouped;     // the others, sorted by (n, shape)
    size_t hdr_off = 0, jobs_off = 0, start_off = 0, group_off = 0, bytes = 0;
    int total[kPasses] = {0, 0, 0, 0, 0};
    bool flat = false;            // one workgroup per item instead of persistent workgroups
};
size_t batch_image_bytes(const std::vector<BatchMember> &m);
// host copy of the image for the device buffer at dev_base (its pointers
// point into that buffer); the persistent counters are zero in it
void build_batch_image(const std::vector<BatchMember> &m, bool f32, unsigned char *dev_base, BatchImage *img,
                       std::vector<unsigned char> &host);
// the passes of an uploaded image; reset: clear the counters with a kernel
// first (graph replays)
hipError_t launch_batch_image(const std::vector<BatchMember> &m, const BatchImage &img, bool f32,
                              unsigned char *dev_base, bool reset, hipStream_t st);
void free_workspace(Workspace *w);
inline size_t spectrum_bytes(int n) { return 8 * (size_t)(n + 1) * (n + 1) * pitch_for(n); }
// the multiplier octant of a grid: (n2 + 1) x pitch(n3) x (n1 + 1) doubles
inline size_t spectrum_bytes_dims(const Dims &d) { return 8 * (size_t)(d.n1 + 1) * (d.n2 + 1) * pitch_for(d.n3); }

}  // namespace psp

struct psp_plan {
    int n = 0;
    double h = 0, L = 0, eps = 0, delta = 0;   // h, L: axis 1
    double hs[3] = {0, 0, 0}, Ls[3] = {0, 0, 0};  // per axis (rectangular box)
    int ns[3] = {0, 0, 0};                         // points per axis
    bool grid = false;                             // unequal point counts per axis
    const psp::Twiddles *tws[3] = {nullptr, nullptr, nullptr};   // per axis (grid)
    int R = 0;
    psp_dtype dtype = PSP_F64;
    std::vector<double> omega, alpha;   // S0
    int device = -1;
    std::shared_ptr<psp::DevSpectrum> spec;
    const psp::Twiddles *tw = nullptr;
    bool precomputed = false;
    // per-stream workspaces and profiling state change under const solves
    // (the solve entry points take const plans): guarded by mu
    mutable std::mutex mu;
    mutable std::map<hipStream_t, psp::Workspace> ws;   // one workspace per stream
    int chunk_tiles = 0;                        // H2-H4 chunking (0: one chunk)
    int i1_group = 0;                           // H1-H2 / H4-H5 i1 grouping (0: none)
    psp::Shape shape;                           // launch shape of the passes
    // per-pass profiling: prof_nev events (and launch-to-pass ids) per solve
    mutable std::vector<hipEvent_t> prof_ev;
    mutable std::vector<int> prof_pass;
    mutable int prof_cap = 0, prof_used = 0, prof_nev = 0;
};

namespace psp {
psp_status check_create(int n, double h, int R, double eps, double delta);
// the process-wide tuned launch shape for (n, tier); the default shape if none
Shape tuned_shape(int n, bool f32);
psp_status plan_workspace(const psp_plan *p, hipStream_t st, Workspace **out);
SolveArgs solve_args(const psp_plan *p, const Workspace &w, const void *rho, void *u);
}  // namespace psp
