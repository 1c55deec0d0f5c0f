// persist.hpp - persistent batched pass kernels.  One launch per pass covers
// every solve of a batch whatever its n (padded length N <= 256); each
// workgroup of PB_THREADS threads takes work items from an atomic counter
// until the pass has none left.  A work item of a strided pass is W =
// PB_THREADS / TPC consecutive columns of the flattened (row, k3) index, so
// small grids fill whole workgroups; a line item is Q = PB_THREADS / TPC
// lines.  Each column or line runs exactly the arithmetic of the per-size
// kernels (same Engine, same radix plan, no automatic contraction), so a
// solve gives bitwise the same result here as alone.
#pragma once
#include "passes.hpp"

namespace psp {

// PJob and PBatch (the device batch image) are declared in kernels.h.

template <int N, int PV> struct PBCfg {
    static constexpr int TPC = N / MaxRadix<N, PV>::value();
    static_assert(PB_THREADS % TPC == 0, "threads per column must divide the workgroup");
    static constexpr int W = PB_THREADS / TPC;   // columns (strided) or lines (line passes) per item
    static constexpr int LINE = N + N / 8;
};

// LDS elements the passes need at most (over N <= 256, max radix 8)
constexpr int PB_LINE_ELEMS = PB_THREADS * 8 * 9 / 8;   // Q * LINE = 432 * max radix
constexpr int PB_STRIDED_ELEMS = PB_THREADS * 8;        // N * W = 384 * max radix

// LDS of the persistent passes, one array per pass family (static: one pair
// per translation unit, i.e. per precision).  The pass bodies below are not
// inlined (each gets its own register allocation instead of the union of
// eleven sizes) and name these arrays directly, so their LDS accesses stay
// LDS instructions.
#ifndef PB_LDS_ELEM
#define PB_LDS_ELEM double2   // the complex type of the including precision
#endif
static __shared__ __attribute__((aligned(16))) PB_LDS_ELEM pb_lds_line[PB_LINE_ELEMS];
static __shared__ __attribute__((aligned(16))) PB_LDS_ELEM pb_lds_strided[PB_STRIDED_ELEMS];

template <typename T> __device__ __forceinline__ Twiddle<T> pb_twiddle(const PJob &jb) {
    Twiddle<T> tw;
    tw.w = (const double2 *)jb.tw64;
    return tw;
}
// the strided passes' twiddles, the same values as the per-size kernels
// read: FP64 roots straight from the global table (the per-size kernels read
// a copy of it in LDS), FP32 the trees (rounding to the same floats)
template <typename T, int N> struct PbStridedTw { using type = Twiddle<T>; };
template <int N> struct PbStridedTw<double, N> { using type = TableTwiddle<double, N>; };
template <typename T, int N> __device__ __forceinline__ typename PbStridedTw<T, N>::type pb_strided_twiddle(const PJob &jb) {
    if constexpr (std::is_same<T, double>::value)
        return TableTwiddle<double, N>{(const double2 *)jb.tw64};
    else
        return pb_twiddle<T>(jb);
}

// ------------------------------------------------------------------- H1
template <typename T, int N, int PV>
__device__ __noinline__ void pb_z_r2c(const PJob *jp, int item) {
    using C = cplx<T>;
    const PJob jb = *jp;
    C *lds = reinterpret_cast<C *>(pb_lds_line);
    using Cfg = PBCfg<N, PV>;
    using E = Engine<T, N, Cfg::TPC, false, PV>;
    constexpr int n = N / 2, Q = Cfg::W;
    const Twiddle<T> tw = pb_twiddle<T>(jb);
    const int t = threadIdx.x % Cfg::TPC, q = threadIdx.x / Cfg::TPC;
    const int pair = item * Q + q;
    const bool active = pair < n * n / 2;
    const T *ra = (const T *)jb.rho + (size_t)(2 * pair) * n;
    const T *rb = ra + n;
    C v[E::V];
    E::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < E::R(0) / 2 && active) return C{g_load(&ra[pos]), g_load(&rb[pos])};
        return c_zero<C>();
    });
    IdxLine idx{q * Cfg::LINE};
    E::template run_from<0>(v, lds, t, idx, tw);
    E::for_outputs(v, t, [&](int pos, int, C &val) { lds[idx(pos)] = val; });
    __syncthreads();
    if (active) {
        C *xa = (C *)jb.X + (size_t)(2 * pair) * jb.P;
        C *xb = xa + jb.P;
        for (int k = t; k <= n; k += Cfg::TPC) {
            const C z = lds[idx(k)];
            const C zc = lds[idx(k == 0 ? 0 : N - k)];
            g_store(&xa[k], C{T(0.5) * (z.x + zc.x), T(0.5) * (z.y - zc.y)});
            const C d = C{z.x - zc.x, z.y + zc.y};
            g_store(&xb[k], C{T(0.5) * d.y, -T(0.5) * d.x});
        }
    }
}

// ------------------------------------------------------------------- H2
// item columns f = item * W + col of the flattened (i1, k3) index
template <typename T, int N, int PV>
__device__ __noinline__ void pb_y_fwd(const PJob *jp, int item) {
    using C = cplx<T>;
    const PJob jb = *jp;
    C *lds = reinterpret_cast<C *>(pb_lds_strided);
    using Cfg = PBCfg<N, PV>;
    using E = Engine<T, N, Cfg::TPC, false, PV>;
    constexpr int n = N / 2, W = Cfg::W;
    const auto tw = pb_strided_twiddle<T, N>(jb);
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int f = item * W + col;
    const int i1 = f / (n + 1), c = f % (n + 1);
    const bool valid = i1 < n;
    const C *src = (const C *)jb.X + (size_t)i1 * n * jb.P + c;
    C *dst = (C *)jb.A + (size_t)i1 * jb.plane + c;
    C v[E::V];
    E::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < E::R(0) / 2 && valid) return g_load(&src[(size_t)pos * jb.P]);
        return c_zero<C>();
    });
    E::template run_from<0>(v, lds, t, IdxInter<W>{col}, tw);
    E::for_outputs(v, t, [&](int pos, int, C &val) {
        if (valid) g_store(&dst[(size_t)pos * jb.pa], val);
    });
}

// ------------------------------------------------------------------- H3
// item columns f of the flattened (k2, k3) index
template <typename T, int N, int PV>
__device__ __noinline__ void pb_x_fused(const PJob *jp, int item) {
    using C = cplx<T>;
    const PJob jb = *jp;
    C *lds = reinterpret_cast<C *>(pb_lds_strided);
    using Cfg = PBCfg<N, PV>;
    using EF = Engine<T, N, Cfg::TPC, false, PV>;
    using EI = Engine<T, N, Cfg::TPC, true, PV>;
    constexpr int n = N / 2, W = Cfg::W;
    const auto tw = pb_strided_twiddle<T, N>(jb);
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int f = item * W + col;
    const int k2 = f / (n + 1), c = f % (n + 1);
    const bool valid = k2 < N;
    const int b = !valid ? 0 : (k2 <= n ? k2 : N - k2);
    const C *src = (const C *)jb.A + (size_t)k2 * jb.pa + c;      // rows i1
    const size_t step = (size_t)jb.plane;
    const double *mrow = jb.mult + ((size_t)(b * (jb.P / 8) + c / 8) * (n + 1)) * 8 + (c & 7);
    C v[EF::V];
    EF::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < EF::R(0) / 2 && valid) return g_load(&src[pos * step]);
        return c_zero<C>();
    });
    EF::template run_from<0>(v, lds, t, IdxInter<W>{col}, tw);
    EF::for_outputs(v, t, [&](int pos, int, C &val) {
        const int a = pos <= n ? pos : N - pos;
        val = scale_mode(val, valid ? g_load(&mrow[(size_t)a * 8]) : 0.0);
    });
    EI::template run_from<0>(v, lds, t, IdxInter<W>{col}, tw);
    C *dst = (C *)jb.A + (size_t)k2 * jb.pa + c;
    EI::for_outputs(v, t, [&](int pos, int r, C &val) {
        if (valid && r < EI::R(EI::S - 1) / 2) g_store(&dst[pos * step], val);
    });
}

// ------------------------------------------------------------------- H4
// item columns f of the flattened (i1, k3) index
template <typename T, int N, int PV>
__device__ __noinline__ void pb_y_inv(const PJob *jp, int item) {
    using C = cplx<T>;
    const PJob jb = *jp;
    C *lds = reinterpret_cast<C *>(pb_lds_strided);
    using Cfg = PBCfg<N, PV>;
    using E = Engine<T, N, Cfg::TPC, true, PV>;
    constexpr int n = N / 2, W = Cfg::W;
    const auto tw = pb_strided_twiddle<T, N>(jb);
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int f = item * W + col;
    const int i1 = f / (n + 1), c = f % (n + 1);
    const bool valid = i1 < n;
    const C *src = (const C *)jb.A + (size_t)i1 * jb.plane + c;   // rows k2
    C v[E::V];
    E::for_inputs(v, t, [&](int pos, int) -> C {
        if (valid) return g_load(&src[(size_t)pos * jb.pa]);
        return c_zero<C>();
    });
    E::template run_from<0>(v, lds, t, IdxInter<W>{col}, tw);
    C *dst = (C *)jb.X + (size_t)i1 * n * jb.P + c;
    E::for_outputs(v, t, [&](int pos, int r, C &val) {
        if (valid && r < E::R(E::S - 1) / 2) g_store(&dst[(size_t)pos * jb.P], val);
    });
}

// ------------------------------------------------------------------- H5
template <typename T, int N, int PV>
__device__ __noinline__ void pb_z_c2r(const PJob *jp, int item) {
    using C = cplx<T>;
    const PJob jb = *jp;
    C *lds = reinterpret_cast<C *>(pb_lds_line);
    using Cfg = PBCfg<N, PV>;
    using E = Engine<T, N, Cfg::TPC, true, PV>;
    constexpr int n = N / 2, Q = Cfg::W;
    const Twiddle<T> tw = pb_twiddle<T>(jb);
    const int t = threadIdx.x % Cfg::TPC, q = threadIdx.x / Cfg::TPC;
    const int pair = item * Q + q;
    const bool active = pair < n * n / 2;
    const C *ya = (const C *)jb.X + (size_t)(2 * pair) * jb.P;
    const C *yb = ya + jb.P;
    IdxLine idx{q * Cfg::LINE};
    constexpr int KB = (n + 1 + Cfg::TPC - 1) / Cfg::TPC;   // bins per thread
    C ba[KB], bb[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        const int k = t + i * Cfg::TPC;
        if (active && k <= n) {
            ba[i] = g_load(&ya[k]);
            bb[i] = g_load(&yb[k]);
        }
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        const int k = t + i * Cfg::TPC;
        if (active && k <= n) {
            C A = ba[i], B = bb[i];
            if (k == 0 || k == n) {
                A.y = 0;
                B.y = 0;
            }
            lds[idx(k)] = C{A.x - B.y, A.y + B.x};
            if (k != 0 && k != n) lds[idx(N - k)] = C{A.x + B.y, B.x - A.y};
        }
    }
    __syncthreads();
    C v[E::V];
    E::template load_lds<0>(v, lds, t, idx);
    __syncthreads();
    E::template run_from<0>(v, lds, t, idx, tw);
    T *ua = (T *)jb.u + (size_t)(2 * pair) * n;
    T *ub = ua + n;
    E::for_outputs(v, t, [&](int pos, int r, C &val) {
        if (active && r < E::R(E::S - 1) / 2) {
            g_store(&ua[pos], val.x);
            g_store(&ub[pos], val.y);
        }
    });
}

// ------------------------------------------------------------- dispatch
template <typename T, int PASS, int N, int PV>
__device__ __forceinline__ void pb_run(const PJob *jp, int item) {
    if constexpr (PASS == 0) pb_z_r2c<T, N, PV>(jp, item);
    else if constexpr (PASS == 1) pb_y_fwd<T, N, PV>(jp, item);
    else if constexpr (PASS == 2) pb_x_fused<T, N, PV>(jp, item);
    else if constexpr (PASS == 3) pb_y_inv<T, N, PV>(jp, item);
    else pb_z_c2r<T, N, PV>(jp, item);
}

template <typename T, int PASS>
__device__ __forceinline__ void pb_dispatch(const PJob *jp, int N, int pv, int item) {
    switch (N) {
#define PSP_PB(NN)                                                              \
    case NN:                                                                    \
        static_assert(MaxRadix<NN, 0>::value() <= 8 &&                          \
                          MaxRadix<NN, alt_plan_exists(NN) ? 1 : 0>::value() <= 8, \
                      "persistent bodies hold radices up to 8: plans 0 and 1");  \
        if (alt_plan_exists(NN) && pv == 1)                                     \
            pb_run<T, PASS, NN, alt_plan_exists(NN) ? 1 : 0>(jp, item);    \
        else                                                                    \
            pb_run<T, PASS, NN, 0>(jp, item);                              \
        break;
        PSP_PB(8) PSP_PB(12) PSP_PB(16) PSP_PB(24) PSP_PB(32) PSP_PB(48) PSP_PB(64) PSP_PB(96)
        PSP_PB(128) PSP_PB(192) PSP_PB(256)
#undef PSP_PB
        default: break;
    }
}

// One pass over every solve of the batch.  Every workgroup leaves once the
// counter passes the pass's total, so the grid always drains.  The item
// offsets of up to PB_CACHED_JOBS jobs are kept in LDS for the job lookup,
// and thread 0 takes the next item from the counter while the current one
// runs, so neither lookup nor counter latency sits between items.  At least
// three waves per SIMD (at most 168 VGPRs): two 6-wave workgroups per CU.
constexpr int PB_CACHED_JOBS = 2048;

template <typename T, int PASS>
__global__ void __launch_bounds__(PB_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_persist(PBatch *bt) {
    __shared__ int s_start[PB_CACHED_JOBS + 1];
    __shared__ int s_next;
    const int total = bt->total[PASS];
    const int njobs = bt->njobs;
    const int *start = bt->start + PASS * (njobs + 1);
    const bool cached = njobs <= PB_CACHED_JOBS;
    if (cached)
        for (int i = threadIdx.x; i <= njobs; i += PB_THREADS) s_start[i] = start[i];
    if (threadIdx.x == 0) s_next = atomicAdd(&bt->counter[PASS], 1);
    __syncthreads();
    for (;;) {
        const int item = s_next;
        __syncthreads();                   // every thread has read s_next
        if (item >= total) break;          // the same value in every thread
        if (threadIdx.x == 0) s_next = atomicAdd(&bt->counter[PASS], 1);
        const int *st = cached ? s_start : start;
        int lo = 0, hi = njobs - 1;        // last job whose first item <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (st[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const PJob *jp = bt->jobs + lo;
        pb_dispatch<T, PASS>(jp, jp->N, jp->pv[PASS], item - st[lo]);
        __syncthreads();                   // LDS reuse; s_next is visible
    }
}

// The same passes with one workgroup per work item (grid = the pass's total):
// still one launch per pass for every solve, with the hardware dispatcher
// instead of the counter handing out items.
template <typename T, int PASS>
__global__ void __launch_bounds__(PB_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_flat(PBatch *bt) {
    const int item = blockIdx.x;
    const int njobs = bt->njobs;
    const int *start = bt->start + PASS * (njobs + 1);
    int lo = 0, hi = njobs - 1;            // last job whose first item <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    const PJob *jp = bt->jobs + lo;
    pb_dispatch<T, PASS>(jp, jp->N, jp->pv[PASS], item - start[lo]);
}

}  // namespace psp
