// spectrum.hip - the kernel-spectrum build (S2) and the host entry points
// that launch the solve passes.
#include <algorithm>

#include "fft_core.hpp"
#include "kernels.h"

namespace psp {

// ------------------------------------------------------------ S2: spectrum
// Vhat[a,b,c] = sum_s w_s (J2(a)J0(b)J0(c) + J0(a)J2(b)J0(c) + J0(a)J0(b)J2(c))
// (the tables of a, b, c from axes 1, 2, 3: the same tables on a cubic box)
// as a GEMM over K = 2R per b: rows a, columns c,
//   Amat[a,(s,0)] = w_s (J2(a)J0(b) + J0(a)J2(b)), Amat[a,(s,1)] = w_s J0(a)J0(b),
//   Bmat[(s,0),c] = J0(c),                       Bmat[(s,1),c] = J2(c),
// on v_mfma_f64_16x16x4_f64 tiles of 16 a x 16 c; the epilogue applies the
// spectral Laplacian, m = scale (w1 a^2 + w2 b^2 + w3 c^2) Vhat with
// w_p = (2 pi/L_p)^2 and scale = -1/(N1 N2 N3).  Octant a <= n1, b <= n2,
// c <= n3 in the layout [b][c/8][a][c%8] (P: the pitch of c).
// Operand layout of the 16x16x4 FP64 MFMA (lane l): A[l%16][l/16],
// B[l/16][l%16], D[l/16 + 4e][l%16] for e < 4.
typedef double v4d __attribute__((ext_vector_type(4)));

// one wave: SPEC_AT 16-row a-tiles for one b against SPEC_CT consecutive
// 16-wide c-tiles (1 x 9: 272 rows and 288 columns for n + 1 = 257); every A
// operand of a k-step feeds SPEC_CT MFMAs and every B operand SPEC_AT, and
// the operands of the next SPEC_PF k-steps (of 4) are in flight while the
// MFMAs of the current one run, so the table loads' latency overlaps the
// matrix work.  Measured on MI355X at n = 256, R = 40 (us per build, the
// result bitwise the same for every choice): 1 x 9 with 2 steps in flight
// 112.5, 3 steps 113.8, 4 steps 140.5; 1 x 6 with 1 step 144, 3 steps 121,
// 5 steps 131, 6 steps 148; 1 x 8 with 4 steps 166; 1 x 17 with 2 or 3
// steps 173; 1 x 4 with 5 steps 182; 2 x 6 with 1 step 171 (244 registers,
// two waves per SIMD)
constexpr int SPEC_AT = 1;
constexpr int SPEC_CT = 9;
constexpr int SPEC_PF = 2;

struct SpecOps {
    double av[SPEC_AT];
    double bv[SPEC_CT];
};

__device__ __forceinline__ void spec_load(SpecOps &o, int k0, int kq, int abase, int b, int cbase, int R,
                                          const SpecTables &tb, const double *__restrict__ omega) {
    const int ks = k0 + kq, s = ks >> 1, ty = ks & 1;
    const bool live = s < R;
    const size_t sr = (size_t)(live ? s : 0);
    const double *j0a = tb.J0[0] + sr * (tb.n[0] + 1), *j2a = tb.J2[0] + sr * (tb.n[0] + 1);
    const double w = live ? omega[s] : 0.0;
    const size_t rb = sr * (tb.n[1] + 1) + b;
    const double j0b = tb.J0[1][rb], j2b = tb.J2[1][rb];
#pragma unroll
    for (int t = 0; t < SPEC_AT; ++t) {
        const int a = abase + t * 16;
        o.av[t] = 0.0;
        if (live && a <= tb.n[0]) o.av[t] = ty == 0 ? w * (j2a[a] * j0b + j0a[a] * j2b) : w * (j0a[a] * j0b);
    }
    const int n = tb.n[2];
    const double *jb = (ty == 0 ? tb.J0[2] : tb.J2[2]) + sr * (n + 1);
#pragma unroll
    for (int q = 0; q < SPEC_CT; ++q) {
        const int c = cbase + q * 16;
        o.bv[q] = (live && c <= n) ? jb[c] : 0.0;
    }
}

__global__ void __launch_bounds__(256)
k_spectrum(SpecTables tb, const double *__restrict__ omega, int R, int P, SpecScale sc,
           double *__restrict__ mult) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nA = tb.n[0], nB = tb.n[1], nC = tb.n[2];
    const int na = ((nA + 1 + 15) / 16 + SPEC_AT - 1) / SPEC_AT, ng = ((nC + 1 + 15) / 16 + SPEC_CT - 1) / SPEC_CT;
    const long item = (long)blockIdx.x * 4 + wave;
    if (item >= (long)(nB + 1) * na * ng) return;   // no barriers in this kernel
    const int b = (int)(item / (na * ng));
    const int rem = (int)(item % (na * ng));
    const int a0 = (rem / ng) * 16 * SPEC_AT, cgrp = (rem % ng) * SPEC_CT;
    const int row = lane & 15, kq = lane >> 4;
    const int n1 = nA + 1;
    const int abase = a0 + row, cbase = cgrp * 16 + row;
    v4d acc[SPEC_AT][SPEC_CT];
#pragma unroll
    for (int t = 0; t < SPEC_AT; ++t)
#pragma unroll
        for (int q = 0; q < SPEC_CT; ++q) acc[t][q] = v4d{0.0, 0.0, 0.0, 0.0};
    // a ring of SPEC_PF k-steps of operands, indexed statically (the loop
    // body covers SPEC_PF steps); step k's slot is refilled with step
    // k + SPEC_PF right after its MFMAs are issued
    SpecOps ops[SPEC_PF];
#pragma unroll
    for (int d = 0; d < SPEC_PF; ++d) spec_load(ops[d], 4 * d, kq, abase, b, cbase, R, tb, omega);
    for (int k0 = 0; k0 < 2 * R; k0 += 4 * SPEC_PF) {
#pragma unroll
        for (int d = 0; d < SPEC_PF; ++d) {
            if (k0 + 4 * d < 2 * R) {
#pragma unroll
                for (int t = 0; t < SPEC_AT; ++t)
#pragma unroll
                    for (int q = 0; q < SPEC_CT; ++q)
                        acc[t][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops[d].av[t], ops[d].bv[q], acc[t][q], 0, 0, 0);
                if (k0 + 4 * (d + SPEC_PF) < 2 * R)
                    spec_load(ops[d], k0 + 4 * (d + SPEC_PF), kq, abase, b, cbase, R, tb, omega);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < SPEC_AT; ++t)
#pragma unroll
        for (int q = 0; q < SPEC_CT; ++q) {
            const int cc = (cgrp + q) * 16 + row;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int aa = a0 + t * 16 + kq + 4 * e;
                if (aa <= nA && cc <= nC) {
                    const double k2 = sc.w[0] * ((double)aa * aa) + sc.w[1] * ((double)b * b) + sc.w[2] * ((double)cc * cc);
                    mult[((size_t)(b * (P / 8) + cc / 8) * n1 + aa) * 8 + (cc & 7)] = sc.scale * k2 * acc[t][q][e];
                }
            }
        }
}

// --------------------------------------------------------------- launchers
static inline int ceil_div_l(long a, long b) { return (int)((a + b - 1) / b); }

hipError_t passes_f64_lo(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);
hipError_t passes_f64_hi(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);
hipError_t passes_f32_lo(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);
hipError_t passes_f32_hi(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);
hipError_t passes_f64_x1(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);
hipError_t passes_f64_x2(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);
hipError_t passes_f32_x1(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);
hipError_t passes_f32_x2(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                         const Shape &sh, bool full, const void *tw64, hipEvent_t *ev,
                         int *ev_pass, int nev, const Dims &dm, int mask, hipStream_t st);

// the instantiation holding padded length N
static auto passes_for(bool f32, int N) {
    if (nine_length(N)) {
        if (f32) return N <= 216 ? passes_f32_x1 : passes_f32_x2;
        return N <= 216 ? passes_f64_x1 : passes_f64_x2;
    }
    if (f32) return N <= 192 ? passes_f32_lo : passes_f32_hi;
    return N <= 192 ? passes_f64_lo : passes_f64_hi;
}

// launches (and so profiling events minus one) of one solve
int solve_launches(int n, bool f32, int chunk_tiles, int i1_group) {
    const int W = strided_width(f32);
    const int ntile = ceil_div_l(n + 1, W);
    const int ct = chunk_tiles > 0 ? std::min(chunk_tiles, ntile) : ntile;
    const int nchunks = ceil_div_l(ntile, ct);
    const bool grouped = nchunks == 1 && i1_group > 0 && i1_group < n;
    if (grouped) return 4 * ceil_div_l(n, i1_group) + 1;
    return 2 + 3 * nchunks;
}

hipError_t launch_solve(const SolveArgs &s, hipStream_t st) {
    const Job one{s.rho, s.u, s.X, s.A, s.mult, s.A2, s.Y2};
    if (s.ns[0] == 0) {
        auto f = passes_for(s.f32, 2 * s.n);
        return f(2 * s.n, one, nullptr, 1, s.P, s.chunk_tiles, s.i1_group, s.shape, s.full, s.tw64, s.ev,
                 s.ev_pass, s.nev, Dims{s.n, s.n, s.n}, 0x1f, st);
    }
    // one pass at a time at the padded length of its axis
    static const int axis_of_pass[5] = {2, 1, 0, 1, 2};
    const Dims dm{s.ns[0], s.ns[1], s.ns[2]};
    for (int p = 0; p < 5; ++p) {
        const int a = axis_of_pass[p], N = 2 * s.ns[a];
        auto f = passes_for(s.f32, N);
        const hipError_t e =
            f(N, one, nullptr, 1, s.P, 0, 0, s.shape, false, s.tw_axis[a], nullptr, nullptr, 0, dm, 1 << p, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_group(int n, bool f32, const Shape &shape, const Job *table_dev, int count, const void *tw64,
                        hipStream_t st) {
    const Job none{};
    const int P = ((n + 1 + 15) / 16) * 16;
    auto f = passes_for(f32, 2 * n);
    return f(2 * n, none, table_dev, count, P, 0, 0, shape, false, tw64, nullptr, nullptr, 0, Dims{n, n, n}, 0x1f,
             st);
}

hipError_t launch_spectrum(const SpecTables &tb, const double *omega, int R, int P, const SpecScale &sc,
                           double *mult, hipStream_t st) {
    const int na = ((tb.n[0] + 1 + 15) / 16 + SPEC_AT - 1) / SPEC_AT;
    const int ng = ((tb.n[2] + 1 + 15) / 16 + SPEC_CT - 1) / SPEC_CT;
    const long items = (long)(tb.n[1] + 1) * na * ng;
    hipLaunchKernelGGL(k_spectrum, dim3(ceil_div_l(items, 4)), dim3(256), 0, st, tb, omega, R, P, sc, mult);
    return hipGetLastError();
}

}  // namespace psp
