// passes.hpp - the solve's device passes and their launch sequence, as
// templates over the precision T and the padded length N; instantiated per
// precision and length range in passes_{f64,f32}_{lo,hi}.hip.
//
// Data layout in HBM for one solve with n points per axis, N = 2n, and
// P = round_up(n+1, 16) (pitch of the half-spectrum axis k3 = 0..n):
//   rho, u : n*n*n real, [i1][i2][i3]
//   X      : n*n*P complex, [i1][i2][k3]   after H1; reused as Y after H4
//   A      : n planes of N rows of pa complex, [i1][k2][k3] after H2; H3
//            updates it in place (pa = the k3 columns of one chunk, a
//            multiple of the row tile; plane pitch a_plane(n, n, pa) >= N pa)
//   mult   : (n+1)*P*(n+1) FP64, blocked [b][c/8][a][c%8] holding the
//            multiplier m(|k1| = a, |k2| = b, k3 = c), zero for c > n
// Passes (Algorithm 2):
//   H1 k_z_r2c   : forward transform along i3 of the padded real lines, two
//                  real lines per complex transform, n+1 bins kept
//   H2 k_y_fwd   : forward along i2 (input rows i2 >= n are zero)
//   H3 k_x_fused : forward along i1 (inputs i1 >= n zero), multiply by m,
//                  inverse along i1 keeping outputs i1 < n
//   H4 k_y_inv   : inverse along k2 keeping outputs i2 < n
//   H5 k_z_c2r   : inverse Hermitian transform along k3 keeping i3 < n
// Every kernel takes its radix plan PV and its tile shape (columns W or
// threads THR per workgroup) as template parameters; the launch sequence
// picks them per pass from a Shape.
#pragma once
#include <algorithm>
#include <type_traits>

#include "fft_core.hpp"
#include "kernels.h"

namespace psp {

// ------------------------------------------------------------ configuration
// k3 columns of one 128-byte row tile of X and A
template <typename T> struct LayoutTile;
template <> struct LayoutTile<double> { static constexpr int W = 8; };
template <> struct LayoutTile<float> { static constexpr int W = 16; };

// strided passes: W columns per workgroup, TPC threads per column.  XCH:
// how values move between FFT stages: 0 through an LDS buffer of all N x W
// positions; 1 in two phases by position half (half the LDS, a staging copy
// in registers); 2 in two phases by column half (half the LDS, no staging).
// HALF: half the threads per column, each with twice the butterflies of a
// stage (fewer waves, more independent work per wave).
template <typename T, int N, int PV, int W, int XCH_ = 0, bool HALF = false> struct StridedCfg {
    static constexpr int TPC1 = N / MaxRadix<N, PV>::value();
    static constexpr int TPC0 = (HALF && TPC1 >= 2) ? TPC1 / 2 : TPC1;
    static constexpr int TPC = (TPC0 * W > 1024) ? TPC0 / 2 : TPC0;
    static constexpr int THREADS = TPC * W;
    static constexpr int XCH = XCH_;
    static constexpr int LDS_ELEMS = XCH ? N * W / 2 : N * W;
    static constexpr int SUB = LayoutTile<T>::W / W;     // workgroups per row tile
};

// line passes: Q complex lines per workgroup of about THR threads
template <typename T, int N, int PV, int THR> struct LineCfg {
    static constexpr int TPC = N / MaxRadix<N, PV>::value();
    static constexpr int Q = (THR / TPC) > 0 ? (THR / TPC) : 1;
    static constexpr int THREADS = TPC * Q;
    static constexpr int LINE = N + N / 8;                          // padded line in LDS
};

template <int W> struct IdxInter {   // (position, column) -> position*W + column
    int col;
    __device__ __forceinline__ int operator()(int pos) const { return pos * W + col; }
};
struct IdxLine {                     // column-major, one padding slot per 8 positions
    int base;
    __device__ __forceinline__ int operator()(int pos) const { return base + pos + (pos >> 3); }
};

// Plain accesses to the solve's buffers, all global memory, made through
// global-address-space pointers.  A pointer read from a job table is generic
// to the compiler, which then emits flat instructions; a flat load in flight
// also holds the LDS wait counter, so each LDS exchange after it waited for
// the load's HBM latency as well.
template <typename C> struct VecOf;
template <> struct VecOf<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float2> { typedef float type __attribute__((ext_vector_type(2))); };
template <typename T> struct GlobalRep { using type = T; };
template <> struct GlobalRep<double2> { using type = VecOf<double2>::type; };
template <> struct GlobalRep<float2> { using type = VecOf<float2>::type; };
template <typename T> __device__ __forceinline__ T g_load(const T *p) {
    using V = typename GlobalRep<T>::type;
    const V t = *(const __attribute__((address_space(1))) V *)p;
    if constexpr (std::is_same<V, T>::value)
        return t;
    else
        return T{t.x, t.y};
}
template <typename T> __device__ __forceinline__ void g_store(T *p, const T &v) {
    using V = typename GlobalRep<T>::type;
    if constexpr (std::is_same<V, T>::value) {
        *(__attribute__((address_space(1))) V *)p = v;
    } else {
        V t;
        t.x = v.x;
        t.y = v.y;
        *(__attribute__((address_space(1))) V *)p = t;
    }
}

// The twiddle source of a pass kernel (STRIDED: H2-H4, else H1/H5): a copy of
// the roots in the workgroup's LDS for the strided passes of both tiers and
// for FP32 line passes of at least 256 threads (tw_lds_elems more elements at
// the end of the kernel's LDS array), else the FP64 power trees: FP64 line
// passes (every shape of a pass reads the same twiddles, so every shape gives
// bitwise the same result) and small FP32 line workgroups, for which the copy
// costs more than the trees.
//
// The copy takes two calls that every thread of the workgroup makes:
// tw_fetch, which issues the global loads of the thread's roots into
// registers, and tw_commit, which stores them to LDS and (SYNC) ends with the
// workgroup barrier.  H1, H3 and H5 issue their own input loads between the
// two, so that the latencies of the table and of the inputs overlap instead
// of following one another; H2 and H4 commit before their loads, which
// measured 3-4 us faster for them at n = 256.  Where a thread would hold
// more than kTwRegs roots the fetch is empty and the commit copies the table
// in a loop.
constexpr int kTwRegs = 4;
template <typename T, int THREADS, bool STRIDED> constexpr bool tw_in_lds() {
    return std::is_same<T, float>::value ? (STRIDED || THREADS >= 256) : STRIDED;
}
template <typename T, int NN, int THREADS, bool STRIDED> constexpr int tw_lds_elems() {
    return tw_in_lds<T, THREADS, STRIDED>() ? NN : 0;
}
template <typename T, int NN, int THREADS, bool STRIDED> struct TwFetch {
    static constexpr int K = tw_in_lds<T, THREADS, STRIDED>() ? (NN + THREADS - 1) / THREADS : 0;
    static constexpr bool REGS = K > 0 && K <= kTwRegs;
    double2 w[REGS ? K : 1];
};
template <typename T, int NN, bool LDS> struct PassTwiddle { using type = Twiddle<T>; };
template <typename T, int NN> struct PassTwiddle<T, NN, true> { using type = TableTwiddle<T, NN>; };
template <typename T, int NN, int THREADS, bool STRIDED>
__device__ __forceinline__ TwFetch<T, NN, THREADS, STRIDED> tw_fetch(const Twiddle<T> &tw) {
    using F = TwFetch<T, NN, THREADS, STRIDED>;
    F f;
    if constexpr (F::REGS) {
#pragma unroll
        for (int k = 0; k < F::K; ++k) {
            const int e = (int)threadIdx.x + k * THREADS;
            if (NN % THREADS == 0 || e < NN) f.w[k] = g_load(&tw.w[e]);
        }
    }
    return f;
}
template <typename T, int NN, int THREADS, bool STRIDED, bool SYNC = true>
__device__ __forceinline__ typename PassTwiddle<T, NN, tw_in_lds<T, THREADS, STRIDED>()>::type
tw_commit(const Twiddle<T> &tw, const TwFetch<T, NN, THREADS, STRIDED> &f, cplx<T> *buf) {
    using F = TwFetch<T, NN, THREADS, STRIDED>;
    if constexpr (tw_in_lds<T, THREADS, STRIDED>()) {
        if constexpr (F::REGS) {
#pragma unroll
            for (int k = 0; k < F::K; ++k) {
                const int e = (int)threadIdx.x + k * THREADS;
                if (NN % THREADS == 0 || e < NN) buf[e] = cplx<T>{T(f.w[k].x), T(f.w[k].y)};
            }
        } else {
            for (int e = threadIdx.x; e < NN; e += THREADS) {
                const double2 w = g_load(&tw.w[e]);
                buf[e] = cplx<T>{T(w.x), T(w.y)};
            }
        }
        if constexpr (SYNC) __syncthreads();
        return TableTwiddle<T, NN>{buf};
    } else {
        (void)f;
        (void)buf;
        return tw;
    }
}

// The multiply of H3: a mode times its FP64 multiplier entry, in FP64 for the
// FP64 tier; for the FP32 tier the entry is rounded once to FP32 and the
// product taken in FP32 (one conversion and two FP32 products per mode
// instead of four conversions and two FP64 products; the rounding of the
// entry adds at most one FP32 unit to the product's own).
__device__ __forceinline__ double2 scale_mode(double2 v, double m) { return double2{v.x * m, v.y * m}; }
__device__ __forceinline__ float2 scale_mode(float2 v, double m) {
    const float mf = (float)m;
    return float2{v.x * mf, v.y * mf};
}

// the FFT stages of a strided pass with the configuration's exchange
template <typename E, typename Cfg, int W, typename C, typename TW>
__device__ __forceinline__ void strided_stages(C *v, C *lds, int t, int col, const TW &tw) {
    if constexpr (Cfg::XCH == 2)
        E::template run_from_cols<0>(v, lds, t, IdxInter<W / 2>{col % (W / 2)}, tw, col < W / 2);
    else
        E::template run_from<0, Cfg::XCH == 1>(v, lds, t, IdxInter<W>{col}, tw);
}

// Per-solve device pointers.  A single solve passes them as a kernel
// argument; a batched launch passes a device table and takes entry
// blockIdx.y (every solve of one launch has the same padded length).
struct JobRef {
    Job arg;
    const Job *table;
    __device__ __forceinline__ Job get() const { return table ? table[blockIdx.y] : arg; }
};

// Cache policy CP of a pass's global accesses: 0 ordinary, 1 nontemporal
// stores, 2 nontemporal loads and stores.  The streaming hints
// let the rows a workgroup touches (128 bytes each, a plane or a row pitch
// apart) go to and come from HBM in the order the workgroups issue them
// instead of as scattered L2 evictions.  They also change the pass after:
// at n = 256 FP64, H5 ran 10 us slower after H4 with nontemporal A loads and
// ordinary X stores, and 12 us faster after H4 with both nontemporal, than
// after an ordinary H4.  In H3 they also keep the stream of A from
// displacing the multiplier blocks the paired workgroups share in L2.  Which one pays
// depends on the size and tier, so it is a tuning choice (H1, H2, H5: 0 or
// 1, H3: 0, 1 or 2, H4: 0 or 2).  The pointers are global memory.
template <int CP, typename C> __device__ __forceinline__ C a_load(const C *p) {
    if constexpr (CP == 2) {
        typedef const __attribute__((address_space(1))) typename VecOf<C>::type *G;
        const auto t = __builtin_nontemporal_load((G)p);
        return C{t.x, t.y};
    } else {
        return g_load(p);
    }
}
template <int CP, typename C> __device__ __forceinline__ void a_store(C *p, const C &v) {
    if constexpr (CP >= 1) {
        typedef __attribute__((address_space(1))) typename VecOf<C>::type *G;
        typename VecOf<C>::type t;
        t.x = v.x;
        t.y = v.y;
        __builtin_nontemporal_store(t, (G)p);
    } else {
        g_store(p, v);
    }
}
template <int CP, typename T> __device__ __forceinline__ void s_store(T *p, T v) {
    if constexpr (CP >= 1) {
        __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T *)p);
    } else {
        g_store(p, v);
    }
}

// ------------------------------------------------------------------- H1
// Two real lines a, b (flattened (i1, i2) = 2q, 2q+1) form z = a + i b.  The
// padded length-N line has data in [0, n) only.  After the transform,
// A[k] = (Z[k] + conj Z[N-k])/2 and B[k] = (Z[k] - conj Z[N-k])/(2i).
template <typename T, int N, int PV, int THR, int CP>
__global__ void __launch_bounds__((LineCfg<T, N, PV, THR>::THREADS))
k_z_r2c(JobRef jr, int npairs, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = LineCfg<T, N, PV, THR>;
    using E = Engine<T, N, Cfg::TPC, false, PV>;
    constexpr int n = N / 2;
    __shared__ C lds[Cfg::Q * Cfg::LINE + tw_lds_elems<T, N, Cfg::THREADS, false>()];
    const auto twf = tw_fetch<T, N, Cfg::THREADS, false>(tw);
    const Job jb = jr.get();
    const int t = threadIdx.x % Cfg::TPC, q = threadIdx.x / Cfg::TPC;
    const int pair = blockIdx.x * Cfg::Q + q;
    const bool active = pair < npairs;
    const T *ra = (const T *)jb.rho + (size_t)(2 * pair) * n;
    const T *rb = ra + n;
    C v[E::V];
    E::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < E::R(0) / 2 && active) return C{g_load(&ra[pos]), g_load(&rb[pos])};
        return c_zero<C>();
    });
    const auto twx = tw_commit<T, N, Cfg::THREADS, false>(tw, twf, lds + Cfg::Q * Cfg::LINE);
    IdxLine idx{q * Cfg::LINE};
    E::template run_from<0>(v, lds, t, idx, twx);
    E::for_outputs(v, t, [&](int pos, int, C &val) { lds[idx(pos)] = val; });
    __syncthreads();
    if (active) {
        C *xa = (C *)jb.X + (size_t)(2 * pair) * P;
        C *xb = xa + P;
        for (int k = t; k <= n; k += Cfg::TPC) {
            const C z = lds[idx(k)];
            const C zc = lds[idx(k == 0 ? 0 : N - k)];
            a_store<CP>(&xa[k], C{T(0.5) * (z.x + zc.x), T(0.5) * (z.y - zc.y)});
            const C d = C{z.x - zc.x, z.y + zc.y};     // Z[k] - conj Z[N-k]
            a_store<CP>(&xb[k], C{T(0.5) * d.y, -T(0.5) * d.x});   // d / (2i)
        }
    }
}

// ------------------------------------------------------------------- H2-H4
// The strided passes work on a chunk of k3 row tiles [tile0, tile0 + ntile)
// (LayoutTile columns each).  The padded intermediate of a chunk is
// A[i1][k2][c] with the chunk-local column c < pa as its contiguous axis
// (measured faster on MI355X than a tile-major layout: the i2 passes then
// touch rows only a few KB apart).  X/Y rows are [i1][i2][k3] with pitch P
// and the global column cg = tile0 * LayoutTile + c, which also decides
// validity (cg <= n) and the multiplier entry.  A workgroup of W columns
// covers 1/SUB of a row tile.
struct Chunk {
    int tile0;      // first row tile of the chunk
    int ntile;      // row tiles in the chunk
    int pa;         // k3 pitch of the chunk buffer A
    int n2;         // points along i2 (rows k2 of A: 2 n2)
    int n3;         // points along i3 (columns k3 <= n3 are valid)
    long long plane;    // i1 pitch of A: a_plane(n1, n2, pa)
};

__device__ __forceinline__ size_t a_index(const Chunk &ck, int c, int k2, int i1) {
    return (size_t)i1 * ck.plane + (size_t)k2 * ck.pa + c;
}

// ------------------------------------------------------------------- H2
template <typename T, int N, int PV, int W, int XC, bool HF, int CP>
__global__ void __launch_bounds__((StridedCfg<T, N, PV, W, XC, HF>::THREADS))
k_y_fwd(JobRef jr, Chunk ck, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = StridedCfg<T, N, PV, W, XC, HF>;
    using E = Engine<T, N, Cfg::TPC, false, PV>;
    constexpr int n = N / 2;
    __shared__ C lds[Cfg::LDS_ELEMS + tw_lds_elems<T, N, Cfg::THREADS, true>()];
    const auto twx = tw_commit<T, N, Cfg::THREADS, true>(tw, tw_fetch<T, N, Cfg::THREADS, true>(tw),
                                                         lds + Cfg::LDS_ELEMS);
    const Job jb = jr.get();
    const int nsub = ck.ntile * Cfg::SUB;
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int i1 = blockIdx.x / nsub, c = (blockIdx.x % nsub) * W + col;
    const int cg = ck.tile0 * LayoutTile<T>::W + c;
    const bool valid = cg <= ck.n3;
    const C *src = (const C *)jb.X + (size_t)i1 * n * P + cg;      // rows i2 of X
    C *dst = (C *)jb.A + a_index(ck, c, 0, i1);                    // rows k2 of A
    C v[E::V];
    E::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < E::R(0) / 2 && valid) return g_load(&src[(size_t)pos * P]);
        return c_zero<C>();
    });
    strided_stages<E, Cfg, W>(v, lds, t, col, twx);
    E::for_outputs(v, t, [&](int pos, int, C &val) { a_store<CP>(&dst[(size_t)pos * ck.pa], val); });
}

// ------------------------------------------------------------------- H3
// Work item (b, sub-tile, side): column k2 = b (side 0) or N - b (side 1),
// both reading the same multiplier block.  Items (b, ., 0) and (b, ., 1) go
// to workgroups g and g + 8, which the dispatcher places on the same XCD at
// nearly the same time, so the second read of the block hits that XCD's L2.
// FULL (test hook): all N outputs of the inverse go to A2[i1][k2][k3] (pitch P).
template <typename T, int N, int PV, int W, int XC, bool HF, bool FULL, int CP>
__global__ void __launch_bounds__((StridedCfg<T, N, PV, W, XC, HF>::THREADS))
k_x_fused(JobRef jr, Chunk ck, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = StridedCfg<T, N, PV, W, XC, HF>;
    using EF = Engine<T, N, Cfg::TPC, false, PV>;
    using EI = Engine<T, N, Cfg::TPC, true, PV>;
    constexpr int n = N / 2;
    __shared__ C lds[Cfg::LDS_ELEMS + tw_lds_elems<T, N, Cfg::THREADS, true>()];
    const int nsub = ck.ntile * Cfg::SUB;
    const int g = blockIdx.x;
    const int pi = (g / 16) * 8 + (g % 8), side = (g % 16) / 8;
    if (pi >= (ck.n2 + 1) * nsub) return;           // uniform over the workgroup
    const int b = pi / nsub, sub = pi % nsub;
    if (side && (b == 0 || b == ck.n2)) return;
    const auto twf = tw_fetch<T, N, Cfg::THREADS, true>(tw);
    const Job jb = jr.get();
    const int k2 = side ? 2 * ck.n2 - b : b;        // rows k2 < 2 n2 of A per i1
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int c = sub * W + col;
    const int cg = ck.tile0 * LayoutTile<T>::W + c;
    const bool valid = cg <= ck.n3;
    // 32-bit byte offsets from the buffers' bases (every buffer of a solve is
    // far below 4 GB): one VALU add per access instead of 64-bit address
    // arithmetic, and the bases stay in scalar registers
    unsigned char *abase = (unsigned char *)jb.A;
    const unsigned acol = (unsigned)(((size_t)k2 * ck.pa + c) * sizeof(C));   // rows i1
    const unsigned astep = (unsigned)((size_t)ck.plane * sizeof(C));
    const unsigned char *mbase = (const unsigned char *)jb.mult;
    const unsigned mcol = (unsigned)((((size_t)(b * (P / 8) + cg / 8) * (n + 1)) * 8 + (cg & 7)) * sizeof(double));
    C v[EF::V];
    EF::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < EF::R(0) / 2 && valid) return a_load<CP>((const C *)(abase + (acol + (unsigned)pos * astep)));
        return c_zero<C>();
    });
    const auto twx = tw_commit<T, N, Cfg::THREADS, true>(tw, twf, lds + Cfg::LDS_ELEMS);
    strided_stages<EF, Cfg, W>(v, lds, t, col, twx);
    EF::for_outputs(v, t, [&](int pos, int r, C &val) {
        // the mode's multiplier row |k1|: for an even last radix, legs below
        // R/2 hold the positions below n and the others those from n up
        constexpr int RL = EF::R(EF::S - 1);
        const int a = (RL % 2 == 0) ? (r < RL / 2 ? pos : N - pos) : (pos <= n ? pos : N - pos);
        val = scale_mode(val, g_load((const double *)(mbase + (mcol + (unsigned)a * (8 * sizeof(double))))));
    });
    strided_stages<EI, Cfg, W>(v, lds, t, col, twx);
    if constexpr (!FULL) {
        EI::for_outputs(v, t, [&](int pos, int r, C &val) {
            if (valid && r < EI::R(EI::S - 1) / 2) a_store<CP>((C *)(abase + (acol + (unsigned)pos * astep)), val);
        });
    } else {
        C *dst = (C *)jb.A2 + (size_t)k2 * P + cg;
        EI::for_outputs(v, t, [&](int pos, int, C &val) {
            if (valid) dst[(size_t)pos * N * P] = val;
        });
    }
}

// ------------------------------------------------------------------- H4
// FULL (test hook): reads A2[i1][k2][k3] for all N rows i1 and writes all N
// outputs to Y2[i1][i2][k3] (pitch P).
template <typename T, int N, int PV, int W, int XC, bool HF, bool FULL, int CP>
__global__ void __launch_bounds__((StridedCfg<T, N, PV, W, XC, HF>::THREADS))
k_y_inv(JobRef jr, Chunk ck, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = StridedCfg<T, N, PV, W, XC, HF>;
    using E = Engine<T, N, Cfg::TPC, true, PV>;
    constexpr int n = N / 2;
    __shared__ C lds[Cfg::LDS_ELEMS + tw_lds_elems<T, N, Cfg::THREADS, true>()];
    const auto twx = tw_commit<T, N, Cfg::THREADS, true>(tw, tw_fetch<T, N, Cfg::THREADS, true>(tw),
                                                         lds + Cfg::LDS_ELEMS);
    const Job jb = jr.get();
    const int nsub = ck.ntile * Cfg::SUB;
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int i1 = blockIdx.x / nsub, c = (blockIdx.x % nsub) * W + col;
    const int cg = ck.tile0 * LayoutTile<T>::W + c;
    const bool valid = cg <= ck.n3;
    C v[E::V];
    if constexpr (!FULL) {
        const C *src = (const C *)jb.A + a_index(ck, c, 0, i1);         // rows k2
        E::for_inputs(v, t, [&](int pos, int) -> C {
            if (valid) return a_load<CP>(&src[(size_t)pos * ck.pa]);
            return c_zero<C>();
        });
    } else {
        const C *src = (const C *)jb.A2 + (size_t)i1 * N * P + cg;
        E::for_inputs(v, t, [&](int pos, int) -> C {
            if (valid) return src[(size_t)pos * P];
            return c_zero<C>();
        });
    }
    strided_stages<E, Cfg, W>(v, lds, t, col, twx);
    constexpr int rows_out = FULL ? N : n;
    C *dst = (C *)(FULL ? jb.Y2 : jb.X) + (size_t)i1 * rows_out * P + cg;
    E::for_outputs(v, t, [&](int pos, int r, C &val) {
        if (valid && (FULL || r < E::R(E::S - 1) / 2)) a_store<CP>(&dst[(size_t)pos * P], val);
    });
}

// ------------------------------------------------------------------- H5
// Rows a, b of Y (Hermitian half spectra) form Z[k] = A[k] + i B[k] on the
// full length N; the inverse transform gives a + i b.  The imaginary parts
// of the k = 0 and k = n bins are dropped (real transform).  FULL: rows of
// Y2 (N*N lines) and all N outputs.
template <typename T, int N, int PV, int THR, bool FULL, int CP>
__global__ void __launch_bounds__((LineCfg<T, N, PV, THR>::THREADS))
k_z_c2r(JobRef jr, int npairs, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = LineCfg<T, N, PV, THR>;
    using E = Engine<T, N, Cfg::TPC, true, PV>;
    constexpr int n = N / 2;
    constexpr int len_out = FULL ? N : n;
    __shared__ C lds[Cfg::Q * Cfg::LINE + tw_lds_elems<T, N, Cfg::THREADS, false>()];
    const auto twf = tw_fetch<T, N, Cfg::THREADS, false>(tw);
    const Job jb = jr.get();
    const int t = threadIdx.x % Cfg::TPC, q = threadIdx.x / Cfg::TPC;
    const int pair = blockIdx.x * Cfg::Q + q;
    const bool active = pair < npairs;
    const C *ya = (const C *)(FULL ? jb.Y2 : jb.X) + (size_t)(2 * pair) * P;
    const C *yb = ya + P;
    IdxLine idx{q * Cfg::LINE};
    // each half-spectrum bin is read once (coalesced) and gives
    // Z[k] = A[k] + i B[k] and Z[N-k] = conj A[k] + i conj B[k]; all of a
    // thread's loads are issued before the first LDS write
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
    // the roots go to LDS with the bins; the barrier below covers both
    const auto twx = tw_commit<T, N, Cfg::THREADS, false, false>(tw, twf, lds + Cfg::Q * Cfg::LINE);
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
    E::template run_from<0>(v, lds, t, idx, twx);
    T *ua = (T *)jb.u + (size_t)(2 * pair) * len_out;
    T *ub = ua + len_out;
    E::for_outputs(v, t, [&](int pos, int r, C &val) {
        if (active && (FULL || r < E::R(E::S - 1) / 2)) {
            s_store<CP>(&ua[pos], val.x);
            s_store<CP>(&ub[pos], val.y);
        }
    });
}

// --------------------------------------------------------------- launchers
inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T> static Twiddle<T> twiddle_of(const void *w) {
    Twiddle<T> tw;
    tw.w = (const double2 *)w;
    return tw;
}

// compile-time choices from the run-time Shape entries
template <int N, typename F> inline void with_plan(int pv, F &&f) {
    if constexpr (alt_plan_exists(N)) {
        if (pv == 1) {
            f(std::integral_constant<int, 1>{});
            return;
        }
    }
    if constexpr (r16_plan_exists(N)) {
        if (pv == 2) {
            f(std::integral_constant<int, 2>{});
            return;
        }
    }
    f(std::integral_constant<int, 0>{});
}
template <int W_, int XC_, bool HF_> struct StridedTile {
    static constexpr int W = W_;
    static constexpr int XC = XC_;
    static constexpr bool HF = HF_;
};
template <typename T, typename F> inline void with_cols(int tile, F &&f) {
    constexpr int LW = LayoutTile<T>::W;
    switch (tile) {
        case 1: f(StridedTile<LW / 2, 0, false>{}); break;
        case 2: f(StridedTile<LW, 1, false>{}); break;
        case 3: f(StridedTile<LW, 0, true>{}); break;
        case 4: f(StridedTile<LW, 1, true>{}); break;
        case 5: f(StridedTile<LW, 2, false>{}); break;
        case 6: f(StridedTile<LW, 2, true>{}); break;
        default: f(StridedTile<LW, 0, false>{}); break;
    }
}
// H3's tile choice: the strided tile (tile mod 7) and the cache policy
// (tile / 7)
template <typename T, typename F> inline void with_h3_tile(int tile, F &&f) {
    with_cols<T>(tile % 7, [&](auto w) {
        switch (tile / 7) {
            case 1: f(w, std::integral_constant<int, 1>{}); break;
            case 2: f(w, std::integral_constant<int, 2>{}); break;
            default: f(w, std::integral_constant<int, 0>{}); break;
        }
    });
}
// H2's and H4's tile choice: the strided tile (tile mod 7) and, for tiles
// 7..13, the nontemporal policy NT (H2: its stores, H4: its loads and stores)
template <typename T, int NT, typename F> inline void with_y_tile(int tile, F &&f) {
    with_cols<T>(tile % 7, [&](auto w) {
        if (tile / 7 == 1)
            f(w, std::integral_constant<int, NT>{});
        else
            f(w, std::integral_constant<int, 0>{});
    });
}
// H1's and H5's tile choice: the workgroup size (tile mod 4) and, for tiles
// 4..7, nontemporal stores (H1: of X, H5: of u)
template <typename F> inline void with_threads(int tile, F &&f) {
    auto go = [&](auto thr) {
        if (tile / 4 == 1)
            f(thr, std::integral_constant<int, 1>{});
        else
            f(thr, std::integral_constant<int, 0>{});
    };
    switch (tile % 4) {
        case 1: go(std::integral_constant<int, 128>{}); break;
        case 2: go(std::integral_constant<int, 512>{}); break;
        case 3: go(std::integral_constant<int, 64>{}); break;
        default: go(std::integral_constant<int, 256>{}); break;
    }
}

// the five passes for `count` solves of one padded length: a single solve
// (table == nullptr, pointers in `one`) or a table of `count` jobs.
//   chunk_tiles > 0: H2-H4 over chunks of k3 row tiles (A holds one chunk);
//   i1_group > 0 (single solve, one chunk): H1->H2 and H4->H5 over groups of
//   i1 slabs, X holding one group, so the i3 intermediate of a group is
//   written and read back while it can still sit in the last-level cache.
// Profiling: event i is recorded before launch i (and one after the last);
// ev_pass[i] receives the pass (0..4) of launch i.
// dm: points along i1, i2, i3; only the passes in `mask` (bit p: pass p)
// run, each of them a transform of length N (a cube runs all five at one
// N; otherwise each pass is launched at the length of its own axis: H1, H5
// along i3, H2, H4 along i2, H3 along i1).
template <typename T, int N>
hipError_t passes_impl(const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                       const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                       int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st) {
    constexpr int n = N / 2;
    constexpr int LW = LayoutTile<T>::W;
    const Twiddle<T> tw = twiddle_of<T>(tw64);
    int launch = 0;
    auto mark = [&](int pass) {
        if (ev && launch < nev) {
            (void)hipEventRecord(ev[launch], st);
            if (ev_pass) ev_pass[launch] = pass;
        }
        ++launch;
    };
    const int ntile = ceil_div(dm.n3 + 1, LW);
    const int y = count;
    if (full) {
        // uncropped variant (one chunk, default shape): A2 and Y2 (N x N x P,
        // row layout) receive all N outputs of the inverse transforms
        using SC = StridedCfg<T, N, 0, LW, 0, false>;
        using LC = LineCfg<T, N, 0, 256>;
        const JobRef jr{one, table};
        const Chunk ck{0, ntile, ntile * LW, n, n, (long long)a_plane(n, n, ntile * LW, sizeof(cplx<T>))};
        hipLaunchKernelGGL((k_z_r2c<T, N, 0, 256, 0>), dim3(ceil_div(n * n / 2, LC::Q), y), dim3(LC::THREADS), 0, st,
                           jr, n * n / 2, P, tw);
        hipLaunchKernelGGL((k_y_fwd<T, N, 0, LW, 0, false, 0>), dim3(n * ntile, y), dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        hipLaunchKernelGGL((k_x_fused<T, N, 0, LW, 0, false, true, 0>), dim3(ceil_div((long)(n + 1) * ntile, 8) * 16, y),
                           dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        hipLaunchKernelGGL((k_y_inv<T, N, 0, LW, 0, false, true, 0>), dim3(N * ntile, y), dim3(SC::THREADS), 0, st, jr, ck, P,
                           tw);
        hipLaunchKernelGGL((k_z_c2r<T, N, 0, 256, true, 0>), dim3(ceil_div(N * N / 2, LC::Q), y), dim3(LC::THREADS),
                           0, st, jr, N * N / 2, P, tw);
        return hipGetLastError();
    }
    auto h1 = [&](const JobRef &jr, int npairs) {
        with_plan<N>(sh.plan[0], [&](auto pv) {
            with_threads(sh.tile[0], [&](auto thr, auto cp) {
                constexpr int PV = decltype(pv)::value, THR = decltype(thr)::value, CP = decltype(cp)::value;
                using LC = LineCfg<T, N, PV, THR>;
                hipLaunchKernelGGL((k_z_r2c<T, N, PV, THR, CP>), dim3(ceil_div(npairs, LC::Q), y), dim3(LC::THREADS),
                                   0, st, jr, npairs, P, tw);
            });
        });
    };
    auto h2 = [&](const JobRef &jr, const Chunk &ck, int rows) {
        with_plan<N>(sh.plan[1], [&](auto pv) {
            with_y_tile<T, 1>(sh.tile[1], [&](auto w, auto cp) {
                constexpr int PV = decltype(pv)::value, W = decltype(w)::W;
                constexpr int XC = decltype(w)::XC;
                constexpr bool HF = decltype(w)::HF;
                constexpr int CP = decltype(cp)::value;
                using SC = StridedCfg<T, N, PV, W, XC, HF>;
                hipLaunchKernelGGL((k_y_fwd<T, N, PV, W, XC, HF, CP>), dim3(rows * ck.ntile * SC::SUB, y),
                                   dim3(SC::THREADS), 0, st, jr, ck, P, tw);
            });
        });
    };
    auto h3 = [&](const JobRef &jr, const Chunk &ck) {
        with_plan<N>(sh.plan[2], [&](auto pv) {
            with_h3_tile<T>(sh.tile[2], [&](auto w, auto cp) {
                constexpr int PV = decltype(pv)::value, W = decltype(w)::W;
                constexpr int XC = decltype(w)::XC;
                constexpr bool HF = decltype(w)::HF;
                constexpr int CP = decltype(cp)::value;
                using SC = StridedCfg<T, N, PV, W, XC, HF>;
                hipLaunchKernelGGL((k_x_fused<T, N, PV, W, XC, HF, false, CP>),
                                   dim3(ceil_div((long)(ck.n2 + 1) * ck.ntile * SC::SUB, 8) * 16, y), dim3(SC::THREADS),
                                   0, st, jr, ck, P, tw);
            });
        });
    };
    auto h4 = [&](const JobRef &jr, const Chunk &ck, int rows) {
        with_plan<N>(sh.plan[3], [&](auto pv) {
            with_y_tile<T, 2>(sh.tile[3], [&](auto w, auto cp) {
                constexpr int PV = decltype(pv)::value, W = decltype(w)::W;
                constexpr int XC = decltype(w)::XC;
                constexpr bool HF = decltype(w)::HF;
                constexpr int CP = decltype(cp)::value;
                using SC = StridedCfg<T, N, PV, W, XC, HF>;
                hipLaunchKernelGGL((k_y_inv<T, N, PV, W, XC, HF, false, CP>), dim3(rows * ck.ntile * SC::SUB, y),
                                   dim3(SC::THREADS), 0, st, jr, ck, P, tw);
            });
        });
    };
    auto h5 = [&](const JobRef &jr, int npairs) {
        with_plan<N>(sh.plan[4], [&](auto pv) {
            with_threads(sh.tile[4], [&](auto thr, auto cp) {
                constexpr int PV = decltype(pv)::value, THR = decltype(thr)::value, CP = decltype(cp)::value;
                using LC = LineCfg<T, N, PV, THR>;
                hipLaunchKernelGGL((k_z_c2r<T, N, PV, THR, false, CP>), dim3(ceil_div(npairs, LC::Q), y),
                                   dim3(LC::THREADS), 0, st, jr, npairs, P, tw);
            });
        });
    };
    const int ct = chunk_tiles > 0 ? std::min(chunk_tiles, ntile) : ntile;
    const int nchunks = ceil_div(ntile, ct);
    const int n1 = dm.n1, n2 = dm.n2, n3 = dm.n3;
    const int G = (table == nullptr && nchunks == 1 && i1_group > 0 && i1_group < n1) ? i1_group : n1;
    const int PA = ct * LW;
    const long long plane = (long long)a_plane(n1, n2, PA, sizeof(cplx<T>));
    auto on = [&](int pass) { return (mask >> pass) & 1; };
    // H1 (+ H2 when grouped) per i1 group
    for (int g0 = 0; g0 < n1 && (on(0) || (G < n1 && on(1))); g0 += G) {
        const int gs = std::min(G, n1 - g0);
        Job j = one;
        if (!table) {
            j.rho = (const T *)one.rho + (size_t)g0 * n2 * n3;
            j.A = (cplx<T> *)one.A + (size_t)g0 * plane;
        }
        const JobRef jr{j, table};
        if (on(0)) {
            mark(0);
            h1(jr, gs * n2 / 2);
        }
        if (G < n1 && on(1)) {
            mark(1);
            h2(jr, Chunk{0, ntile, PA, n2, n3, plane}, gs);
        }
    }
    const JobRef jr{one, table};
    for (int ch = 0; ch < nchunks; ++ch) {
        const int t0 = ch * ct, nt = std::min(ct, ntile - t0);
        const Chunk ck{t0, nt, PA, n2, n3, plane};
        if (G == n1 && on(1)) {
            mark(1);
            h2(jr, ck, n1);
        }
        if (on(2)) {
            mark(2);
            h3(jr, ck);
        }
        if (G == n1 && on(3)) {
            mark(3);
            h4(jr, ck, n1);
        }
    }
    // (H4 +) H5 per i1 group
    for (int g0 = 0; g0 < n1 && (on(4) || (G < n1 && on(3))); g0 += G) {
        const int gs = std::min(G, n1 - g0);
        Job j = one;
        if (!table) {
            j.u = (T *)one.u + (size_t)g0 * n2 * n3;
            j.A = (cplx<T> *)one.A + (size_t)g0 * plane;
        }
        const JobRef jrg{j, table};
        if (G < n1 && on(3)) {
            mark(3);
            h4(jrg, Chunk{0, ntile, PA, n2, n3, plane}, gs);
        }
        if (on(4)) {
            mark(4);
            h5(jrg, gs * n2 / 2);
        }
    }
    mark(-1);
    return hipGetLastError();
}

// the pass sequence of one padded length behind a run-time switch; each
// instantiation file covers a subset of the lengths (PSP_CASE per length)
#define PSP_PASSES_SIGNATURE                                                                                  \
    (int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group, const Shape &sh, \
     bool full, const void *tw64, hipEvent_t *ev, int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st)
#define PSP_CASE(T, NN)                                                                                        \
    case NN:                                                                                                   \
        return passes_impl<T, NN>(one, table, count, P, chunk_tiles, i1_group, sh, full, tw64, ev,     \
                                  ev_pass, nev, dm, mask, st);

// padded lengths up to 192 in the *_lo files, the rest in the *_hi files
hipError_t passes_f64_lo PSP_PASSES_SIGNATURE;
hipError_t passes_f64_hi PSP_PASSES_SIGNATURE;
hipError_t passes_f32_lo PSP_PASSES_SIGNATURE;
hipError_t passes_f32_hi PSP_PASSES_SIGNATURE;

}  // namespace psp
