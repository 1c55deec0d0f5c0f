// passes.hip - the solve's device passes and the kernel-spectrum build.
//
// Data layout in HBM for one solve with n points per axis, N = 2n, and
// P = round_up(n+1, 16) (pitch of the half-spectrum axis k3 = 0..n):
//   rho, u : n*n*n real, [i1][i2][i3]
//   X      : n*n*P complex, [i1][i2][k3]   after H1; reused as Y after H4
//   A      : n*N*P complex, [i1][k2][k3]   after H2; H3 updates it in place
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
#include <algorithm>

#include "fft_core.hpp"
#include "kernels.h"

namespace psp {

// ------------------------------------------------------------ configuration
template <typename T> struct StridedCols;
template <> struct StridedCols<double> { static constexpr int W = 8; };   // 128 B rows
template <> struct StridedCols<float> { static constexpr int W = 16; };   // 128 B rows

// occupancy of one workgroup configuration on a CU (160 KB LDS, at most 32
// waves of 64 lanes)
constexpr int wgs_per_cu(int threads, int lds_bytes) {
    const int by_waves = 32 / ((threads + 63) / 64);
    const int by_lds = lds_bytes > 0 ? (160 * 1024) / lds_bytes : by_waves;
    return by_waves < by_lds ? by_waves : by_lds;
}

template <typename T, int N> struct StridedCfg {
    static constexpr int W = StridedCols<T>::W;
    static constexpr int TPC0 = N / MaxRadix<N>::value();
    static constexpr int TPC = (TPC0 * W > 1024) ? TPC0 / 2 : TPC0;
    static constexpr int THREADS = TPC * W;
    static constexpr int FULL_LDS = N * W * (int)sizeof(cplx<T>);
    // exchange through half-size buffers when the LDS, not the wave count,
    // limits how many workgroups share a CU
    // (measured on MI355X: not faster for the FP64 n = 256 passes, so off;
    // PSP_SPLIT_EXCHANGE=1 at build time turns it on where it raises occupancy)
#ifdef PSP_SPLIT_EXCHANGE
    static constexpr bool SPLIT = wgs_per_cu(THREADS, FULL_LDS / 2) > wgs_per_cu(THREADS, FULL_LDS);
#else
    static constexpr bool SPLIT = false;
#endif
    static constexpr int LDS_ELEMS = SPLIT ? N * W / 2 : N * W;
};

template <typename T, int N> struct LineCfg {
    static constexpr int TPC = N / MaxRadix<N>::value();
    static constexpr int Q = (256 / TPC) > 0 ? (256 / TPC) : 1;   // complex lines per WG
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

// Per-solve device pointers.  A single solve passes them as a kernel
// argument; a batched launch passes a device table and takes entry
// blockIdx.y (every solve of one launch has the same padded length).
struct JobRef {
    Job arg;
    const Job *table;
    __device__ __forceinline__ Job get() const { return table ? table[blockIdx.y] : arg; }
};

// ------------------------------------------------------------------- H1
// Two real lines a, b (flattened (i1, i2) = 2q, 2q+1) form z = a + i b.  The
// padded length-N line has data in [0, n) only.  After the transform,
// A[k] = (Z[k] + conj Z[N-k])/2 and B[k] = (Z[k] - conj Z[N-k])/(2i).
template <typename T, int N>
__global__ void __launch_bounds__((LineCfg<T, N>::THREADS))
k_z_r2c(JobRef jr, int npairs, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = LineCfg<T, N>;
    using E = Engine<T, N, Cfg::TPC, false>;
    constexpr int n = N / 2;
    __shared__ C lds[Cfg::Q * Cfg::LINE];
    const Job jb = jr.get();
    const int t = threadIdx.x % Cfg::TPC, q = threadIdx.x / Cfg::TPC;
    const int pair = blockIdx.x * Cfg::Q + q;
    const bool active = pair < npairs;
    const T *ra = (const T *)jb.rho + (size_t)(2 * pair) * n;
    const T *rb = ra + n;
    C v[E::V];
    E::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < E::R(0) / 2 && active) return C{ra[pos], rb[pos]};
        return c_zero<C>();
    });
    IdxLine idx{q * Cfg::LINE};
    E::template run_from<0>(v, lds, t, idx, tw);
    E::for_outputs(v, t, [&](int pos, int, C &val) { lds[idx(pos)] = val; });
    __syncthreads();
    if (active) {
        C *xa = (C *)jb.X + (size_t)(2 * pair) * P;
        C *xb = xa + P;
        for (int k = t; k <= n; k += Cfg::TPC) {
            const C z = lds[idx(k)];
            const C zc = lds[idx(k == 0 ? 0 : N - k)];
            xa[k] = C{T(0.5) * (z.x + zc.x), T(0.5) * (z.y - zc.y)};
            const C d = C{z.x - zc.x, z.y + zc.y};     // Z[k] - conj Z[N-k]
            xb[k] = C{T(0.5) * d.y, -T(0.5) * d.x};   // d / (2i)
        }
    }
}

// ------------------------------------------------------------------- H2-H4
// The strided passes work on a chunk of W-wide k3 tiles [tile0, tile0 +
// ntile).  The padded intermediate of a chunk is A[i1][k2][c] with the
// chunk-local column c < pa = ntile_chunk W as its contiguous axis (measured
// faster on MI355X than a tile-major layout: the i2 passes then touch rows
// only a few KB apart).  X/Y rows are [i1][i2][k3] with pitch P and the
// global column cg = tile0 W + c, which also decides validity (cg <= n) and
// the multiplier entry.
struct Chunk {
    int tile0;      // first tile of the chunk
    int ntile;      // tiles in the chunk
    int pa;         // k3 pitch of the chunk buffer A
};

template <int N, int W>
__device__ __forceinline__ size_t a_index(int pa, int tile, int k2, int i1, int w) {
    return ((size_t)i1 * N + k2) * pa + (size_t)tile * W + w;
}

// ------------------------------------------------------------------- H2
template <typename T, int N>
__global__ void __launch_bounds__((StridedCfg<T, N>::THREADS))
k_y_fwd(JobRef jr, Chunk ck, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = StridedCfg<T, N>;
    using E = Engine<T, N, Cfg::TPC, false>;
    constexpr int n = N / 2, W = Cfg::W;
    __shared__ C lds[Cfg::LDS_ELEMS];
    const Job jb = jr.get();
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int i1 = blockIdx.x / ck.ntile, tile = blockIdx.x % ck.ntile;
    const int cg = (ck.tile0 + tile) * W + col;
    const bool valid = cg <= n;
    const C *src = (const C *)jb.X + (size_t)i1 * n * P + cg;            // rows i2 of X
    C *dst = (C *)jb.A + a_index<N, W>(ck.pa, tile, 0, i1, col);         // rows k2 of A
    C v[E::V];
    E::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < E::R(0) / 2 && valid) return src[(size_t)pos * P];
        return c_zero<C>();
    });
    E::template run_from<0, Cfg::SPLIT>(v, lds, t, IdxInter<W>{col}, tw);
    E::for_outputs(v, t, [&](int pos, int, C &val) { dst[(size_t)pos * ck.pa] = val; });
}

// ------------------------------------------------------------------- H3
// Work item (b, tile, side): column k2 = b (side 0) or N - b (side 1), both
// reading the same multiplier block.  Items (b, tile, 0) and (b, tile, 1) go
// to workgroups g and g + 8, which the dispatcher places on the same XCD at
// nearly the same time, so the second read of the block hits that XCD's L2.
// FULL (test hook): all N outputs of the inverse go to A2[i1][k2][k3] (pitch P).
template <typename T, int N, bool FULL>
__global__ void __launch_bounds__((StridedCfg<T, N>::THREADS))
k_x_fused(JobRef jr, Chunk ck, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = StridedCfg<T, N>;
    using EF = Engine<T, N, Cfg::TPC, false>;
    using EI = Engine<T, N, Cfg::TPC, true>;
    constexpr int n = N / 2, W = Cfg::W;
    __shared__ C lds[Cfg::LDS_ELEMS];
    const int g = blockIdx.x;
    const int pi = (g / 16) * 8 + (g % 8), side = (g % 16) / 8;
    if (pi >= (n + 1) * ck.ntile) return;           // uniform over the workgroup
    const int b = pi / ck.ntile, tile = pi % ck.ntile;
    if (side && (b == 0 || b == n)) return;
    const Job jb = jr.get();
    const int k2 = side ? N - b : b;
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int cg = (ck.tile0 + tile) * W + col;
    const bool valid = cg <= n;
    const C *src = (const C *)jb.A + a_index<N, W>(ck.pa, tile, k2, 0, col);   // rows i1
    const size_t step = (size_t)N * ck.pa;
    const double *mrow = jb.mult + ((size_t)(b * (P / 8) + cg / 8) * (n + 1)) * 8 + (cg & 7);
    C v[EF::V];
    EF::for_inputs(v, t, [&](int pos, int r) -> C {
        if (r < EF::R(0) / 2 && valid) return src[pos * step];
        return c_zero<C>();
    });
    EF::template run_from<0, Cfg::SPLIT>(v, lds, t, IdxInter<W>{col}, tw);
    EF::for_outputs(v, t, [&](int pos, int, C &val) {
        const int a = pos <= n ? pos : N - pos;
        const double m = mrow[(size_t)a * 8];
        val = C{T((double)val.x * m), T((double)val.y * m)};
    });
    EI::template run_from<0, Cfg::SPLIT>(v, lds, t, IdxInter<W>{col}, tw);
    if constexpr (!FULL) {
        C *dst = (C *)jb.A + a_index<N, W>(ck.pa, tile, k2, 0, col);
        EI::for_outputs(v, t, [&](int pos, int r, C &val) {
            if (valid && r < EI::R(EI::S - 1) / 2) dst[pos * step] = val;
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
template <typename T, int N, bool FULL>
__global__ void __launch_bounds__((StridedCfg<T, N>::THREADS))
k_y_inv(JobRef jr, Chunk ck, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = StridedCfg<T, N>;
    using E = Engine<T, N, Cfg::TPC, true>;
    constexpr int n = N / 2, W = Cfg::W;
    __shared__ C lds[Cfg::LDS_ELEMS];
    const Job jb = jr.get();
    const int col = threadIdx.x % W, t = threadIdx.x / W;
    const int i1 = blockIdx.x / ck.ntile, tile = blockIdx.x % ck.ntile;
    const int cg = (ck.tile0 + tile) * W + col;
    const bool valid = cg <= n;
    C v[E::V];
    if constexpr (!FULL) {
        const C *src = (const C *)jb.A + a_index<N, W>(ck.pa, tile, 0, i1, col);   // rows k2
        E::for_inputs(v, t, [&](int pos, int) -> C {
            if (valid) return src[(size_t)pos * ck.pa];
            return c_zero<C>();
        });
    } else {
        const C *src = (const C *)jb.A2 + (size_t)i1 * N * P + cg;
        E::for_inputs(v, t, [&](int pos, int) -> C {
            if (valid) return src[(size_t)pos * P];
            return c_zero<C>();
        });
    }
    E::template run_from<0, Cfg::SPLIT>(v, lds, t, IdxInter<W>{col}, tw);
    constexpr int rows_out = FULL ? N : n;
    C *dst = (C *)(FULL ? jb.Y2 : jb.X) + (size_t)i1 * rows_out * P + cg;
    E::for_outputs(v, t, [&](int pos, int r, C &val) {
        if (valid && (FULL || r < E::R(E::S - 1) / 2)) dst[(size_t)pos * P] = val;
    });
}

// ------------------------------------------------------------------- H5
// Rows a, b of Y (Hermitian half spectra) form Z[k] = A[k] + i B[k] on the
// full length N; the inverse transform gives a + i b.  The imaginary parts
// of the k = 0 and k = n bins are dropped (real transform).  FULL: rows of
// Y2 (N*N lines) and all N outputs.
template <typename T, int N, bool FULL>
__global__ void __launch_bounds__((LineCfg<T, N>::THREADS))
k_z_c2r(JobRef jr, int npairs, int P, Twiddle<T> tw) {
    using C = cplx<T>;
    using Cfg = LineCfg<T, N>;
    using E = Engine<T, N, Cfg::TPC, true>;
    constexpr int n = N / 2;
    constexpr int len_out = FULL ? N : n;
    __shared__ C lds[Cfg::Q * Cfg::LINE];
    const Job jb = jr.get();
    const int t = threadIdx.x % Cfg::TPC, q = threadIdx.x / Cfg::TPC;
    const int pair = blockIdx.x * Cfg::Q + q;
    const bool active = pair < npairs;
    const C *ya = (const C *)(FULL ? jb.Y2 : jb.X) + (size_t)(2 * pair) * P;
    const C *yb = ya + P;
    IdxLine idx{q * Cfg::LINE};
    // each half-spectrum bin is read once (coalesced) and gives
    // Z[k] = A[k] + i B[k] and Z[N-k] = conj A[k] + i conj B[k]
    if (active) {
        for (int k = t; k <= n; k += Cfg::TPC) {
            C A = ya[k], B = yb[k];
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
    T *ua = (T *)jb.u + (size_t)(2 * pair) * len_out;
    T *ub = ua + len_out;
    E::for_outputs(v, t, [&](int pos, int r, C &val) {
        if (active && (FULL || r < E::R(E::S - 1) / 2)) {
            ua[pos] = val.x;
            ub[pos] = val.y;
        }
    });
}

// ------------------------------------------------------------ S2: spectrum
// Vhat[a,b,c] = sum_s w_s (J2(a)J0(b)J0(c) + J0(a)J2(b)J0(c) + J0(a)J0(b)J2(c))
// as a GEMM over K = 2R per b: rows a, columns c,
//   Amat[a,(s,0)] = w_s (J2(a)J0(b) + J0(a)J2(b)), Amat[a,(s,1)] = w_s J0(a)J0(b),
//   Bmat[(s,0),c] = J0(c),                       Bmat[(s,1),c] = J2(c),
// on v_mfma_f64_16x16x4_f64 tiles of 16 a x 16 c; the epilogue applies
// m = scale (a^2 + b^2 + c^2) Vhat with scale = -(2 pi/L)^2 / N^3.
// Operand layout of the 16x16x4 FP64 MFMA (lane l): A[l%16][l/16],
// B[l/16][l%16], D[l/16 + 4e][l%16] for e < 4.
typedef double v4d __attribute__((ext_vector_type(4)));

// one wave: a 16-row a-tile for one b against CT consecutive 16-wide c-tiles;
// the A operand of each k-step is formed once and feeds CT MFMAs
constexpr int SPEC_CT = 4;

__global__ void __launch_bounds__(256)
k_spectrum(const double *__restrict__ J0, const double *__restrict__ J2,
           const double *__restrict__ omega, int R, int n, int P, double scale,
           double *__restrict__ mult) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nt = (n + 1 + 15) / 16, ng = (nt + SPEC_CT - 1) / SPEC_CT;
    const long item = (long)blockIdx.x * 4 + wave;
    if (item >= (long)(n + 1) * nt * ng) return;    // no barriers in this kernel
    const int b = (int)(item / (nt * ng));
    const int rem = (int)(item % (nt * ng));
    const int a0 = (rem / ng) * 16, cgrp = (rem % ng) * SPEC_CT;
    const int row = lane & 15, kq = lane >> 4;
    const int a = a0 + row;
    const int n1 = n + 1;
    v4d acc[SPEC_CT];
#pragma unroll
    for (int q = 0; q < SPEC_CT; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < 2 * R; k0 += 4) {
        const int ks = k0 + kq, s = ks >> 1, ty = ks & 1;
        double av = 0.0;
        const double *j0 = J0 + (size_t)s * n1, *j2 = J2 + (size_t)s * n1;
        if (s < R && a <= n) {
            const double w = omega[s];
            av = ty == 0 ? w * (j2[a] * j0[b] + j0[a] * j2[b]) : w * (j0[a] * j0[b]);
        }
        const double *jb = ty == 0 ? j0 : j2;
#pragma unroll
        for (int q = 0; q < SPEC_CT; ++q) {
            const int c = (cgrp + q) * 16 + row;
            const double bv = (s < R && c <= n) ? jb[c] : 0.0;
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < SPEC_CT; ++q) {
        const int cc = (cgrp + q) * 16 + row;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int aa = a0 + kq + 4 * e;
            if (aa <= n && cc <= n) {
                const double k2 = (double)aa * aa + (double)b * b + (double)cc * cc;
                mult[((size_t)(b * (P / 8) + cc / 8) * n1 + aa) * 8 + (cc & 7)] = scale * k2 * acc[q][e];
            }
        }
    }
}

// --------------------------------------------------------------- launchers
static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

int strided_width(bool f32) { return f32 ? StridedCols<float>::W : StridedCols<double>::W; }

template <typename T, int N> static Twiddle<T> twiddle_of(const void *hi, const void *lo) {
    Twiddle<T> tw;
    if constexpr (sizeof(T) == 8) {
        (void)lo;
        tw.w = (const double2 *)hi;
    } else {
        tw.hi = (const float2 *)hi;
        tw.lo = (const float2 *)lo;
    }
    return tw;
}

// the five passes for `count` solves of one padded length: a single solve
// (table == nullptr, pointers in `one`) or a table of `count` jobs.
//   chunk_tiles > 0: H2-H4 over chunks of k3 tiles (A holds one chunk);
//   i1_group > 0 (single solve, one chunk): H1->H2 and H4->H5 over groups of
//   i1 slabs, X holding one group, so the i3 intermediate of a group is
//   written and read back while it can still sit in the last-level cache.
// Profiling: event i is recorded before launch i (and one after the last);
// ev_pass[i] receives the pass (0..4) of launch i.
template <typename T, int N>
static hipError_t passes_impl(const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                              bool full, const void *tw_hi, const void *tw_lo, hipEvent_t *ev, int *ev_pass, int nev,
                              hipStream_t st) {
    constexpr int n = N / 2;
    const Twiddle<T> tw = twiddle_of<T, N>(tw_hi, tw_lo);
    int launch = 0;
    auto mark = [&](int pass) {
        if (ev && launch < nev) {
            (void)hipEventRecord(ev[launch], st);
            if (ev_pass) ev_pass[launch] = pass;
        }
        ++launch;
    };
    using SC = StridedCfg<T, N>;
    using LC = LineCfg<T, N>;
    constexpr int W = SC::W;
    const int ntile = ceil_div(n + 1, W);
    const int y = count;
    if (full) {
        // uncropped variant (one chunk): A2 and Y2 (N x N x P, row layout)
        // receive all N outputs of the inverse transforms
        const JobRef jr{one, table};
        const Chunk ck{0, ntile, ntile * W};
        hipLaunchKernelGGL((k_z_r2c<T, N>), dim3(ceil_div(n * n / 2, LC::Q), y), dim3(LC::THREADS), 0, st, jr,
                           n * n / 2, P, tw);
        hipLaunchKernelGGL((k_y_fwd<T, N>), dim3(n * ntile, y), dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        hipLaunchKernelGGL((k_x_fused<T, N, true>), dim3(ceil_div((long)(n + 1) * ntile, 8) * 16, y),
                           dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        hipLaunchKernelGGL((k_y_inv<T, N, true>), dim3(N * ntile, y), dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        hipLaunchKernelGGL((k_z_c2r<T, N, true>), dim3(ceil_div(N * N / 2, LC::Q), y), dim3(LC::THREADS), 0, st,
                           jr, N * N / 2, P, tw);
        return hipGetLastError();
    }
    const int ct = chunk_tiles > 0 ? std::min(chunk_tiles, ntile) : ntile;
    const int nchunks = ceil_div(ntile, ct);
    const int G = (table == nullptr && nchunks == 1 && i1_group > 0 && i1_group < n) ? i1_group : n;
    const int PA = ct * W;
    // H1 (+ H2 when grouped) per i1 group
    for (int g0 = 0; g0 < n; g0 += G) {
        const int gs = std::min(G, n - g0);
        Job j = one;
        if (!table) {
            j.rho = (const T *)one.rho + (size_t)g0 * n * n;
            j.A = (cplx<T> *)one.A + (size_t)g0 * N * PA;
        }
        const JobRef jr{j, table};
        mark(0);
        hipLaunchKernelGGL((k_z_r2c<T, N>), dim3(ceil_div(gs * n / 2, LC::Q), y), dim3(LC::THREADS), 0, st, jr,
                           gs * n / 2, P, tw);
        if (G < n) {
            const Chunk ck{0, ntile, PA};
            mark(1);
            hipLaunchKernelGGL((k_y_fwd<T, N>), dim3(gs * ntile, y), dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        }
    }
    const JobRef jr{one, table};
    for (int ch = 0; ch < nchunks; ++ch) {
        const int t0 = ch * ct, nt = std::min(ct, ntile - t0);
        const Chunk ck{t0, nt, PA};
        if (G == n) {
            mark(1);
            hipLaunchKernelGGL((k_y_fwd<T, N>), dim3(n * nt, y), dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        }
        mark(2);
        hipLaunchKernelGGL((k_x_fused<T, N, false>), dim3(ceil_div((long)(n + 1) * nt, 8) * 16, y),
                           dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        if (G == n) {
            mark(3);
            hipLaunchKernelGGL((k_y_inv<T, N, false>), dim3(n * nt, y), dim3(SC::THREADS), 0, st, jr, ck, P, tw);
        }
    }
    // (H4 +) H5 per i1 group
    for (int g0 = 0; g0 < n; g0 += G) {
        const int gs = std::min(G, n - g0);
        Job j = one;
        if (!table) {
            j.u = (T *)one.u + (size_t)g0 * n * n;
            j.A = (cplx<T> *)one.A + (size_t)g0 * N * PA;
        }
        const JobRef jrg{j, table};
        if (G < n) {
            const Chunk ck{0, ntile, PA};
            mark(3);
            hipLaunchKernelGGL((k_y_inv<T, N, false>), dim3(gs * ntile, y), dim3(SC::THREADS), 0, st, jrg, ck, P,
                               tw);
        }
        mark(4);
        hipLaunchKernelGGL((k_z_c2r<T, N, false>), dim3(ceil_div(gs * n / 2, LC::Q), y), dim3(LC::THREADS), 0, st,
                           jrg, gs * n / 2, P, tw);
    }
    mark(-1);
    return hipGetLastError();
}

// launches (and so profiling events minus one) of one solve
int solve_launches(int n, bool f32, int chunk_tiles, int i1_group) {
    const int W = f32 ? StridedCols<float>::W : StridedCols<double>::W;
    const int ntile = ceil_div(n + 1, W);
    const int ct = chunk_tiles > 0 ? std::min(chunk_tiles, ntile) : ntile;
    const int nchunks = ceil_div(ntile, ct);
    const bool grouped = nchunks == 1 && i1_group > 0 && i1_group < n;
    if (grouped) return 4 * ceil_div(n, i1_group) + 1;
    return 2 + 3 * nchunks;
}

template <typename T>
static hipError_t passes_dispatch(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles,
                                  int i1_group, bool full, const void *tw_hi, const void *tw_lo, hipEvent_t *ev,
                                  int *ev_pass, int nev, hipStream_t st) {
    switch (N) {
#define PSP_CASE(NN)                                                                                          \
    case NN:                                                                                                  \
        return passes_impl<T, NN>(one, table, count, P, chunk_tiles, i1_group, full, tw_hi, tw_lo, ev, ev_pass, \
                                  nev, st);
        PSP_CASE(8) PSP_CASE(12) PSP_CASE(16) PSP_CASE(24) PSP_CASE(32) PSP_CASE(48) PSP_CASE(64)
        PSP_CASE(96) PSP_CASE(128) PSP_CASE(192) PSP_CASE(256) PSP_CASE(384) PSP_CASE(512) PSP_CASE(768)
#undef PSP_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve(const SolveArgs &s, hipStream_t st) {
    const Job one{s.rho, s.u, s.X, s.A, s.mult, s.A2, s.Y2};
    return s.f32 ? passes_dispatch<float>(2 * s.n, one, nullptr, 1, s.P, s.chunk_tiles, s.i1_group, s.full, s.tw_hi,
                                          s.tw_lo, s.ev, s.ev_pass, s.nev, st)
                 : passes_dispatch<double>(2 * s.n, one, nullptr, 1, s.P, s.chunk_tiles, s.i1_group, s.full,
                                           s.tw_hi, s.tw_lo, s.ev, s.ev_pass, s.nev, st);
}

hipError_t launch_group(int n, bool f32, const Job *table_dev, int count, const void *tw_hi, const void *tw_lo,
                        hipStream_t st) {
    const Job none{};
    const int P = ((n + 1 + 15) / 16) * 16;
    return f32 ? passes_dispatch<float>(2 * n, none, table_dev, count, P, 0, 0, false, tw_hi, tw_lo, nullptr, nullptr,
                                        0, st)
               : passes_dispatch<double>(2 * n, none, table_dev, count, P, 0, 0, false, tw_hi, tw_lo, nullptr, nullptr,
                                         0, st);
}

hipError_t launch_spectrum(const double *J0, const double *J2, const double *omega, int R, int n, int P,
                           double scale, double *mult, hipStream_t st) {
    const int nt = (n + 1 + 15) / 16, ng = (nt + SPEC_CT - 1) / SPEC_CT;
    const long items = (long)(n + 1) * nt * ng;
    hipLaunchKernelGGL(k_spectrum, dim3(ceil_div(items, 4)), dim3(256), 0, st, J0, J2, omega, R, n, P, scale,
                       mult);
    return hipGetLastError();
}

}  // namespace psp
