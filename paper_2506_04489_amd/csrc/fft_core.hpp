// fft_core.hpp - device building blocks of the solver's FFT passes (gfx950).
//
// Every pass transforms many independent length-N columns (N = 2n, the
// padded length, N = 2^a 3^b) in one workgroup.  A column is processed by
// TPC threads with the Stockham autosort formulation: stage s of radix R
// with Ns = product of the earlier radices maps the butterfly j (0 <= j < N/R)
// from inputs at  j + r N/R  (r < R), twiddled by W_N^{(j mod Ns) r N/(Ns R)},
// to outputs at  (j / Ns) Ns R + (j mod Ns) + r Ns.  Stage data lives in
// registers; the exchange between stages goes through LDS.  The first stage
// reads its inputs straight from global memory, the last stage writes its
// outputs straight to global memory, and (Ns = 1 at the first stage,
// Ns = N/R at the last) both touch positions  j + r N/R  only, which lets a
// pass skip the known-zero half of a zero-padded input, skip the cropped
// half of an output, and run an inverse transform directly on the registers
// a forward transform left behind (the inverse plan is the forward plan in
// reverse order).
#pragma once
#include <hip/hip_runtime.h>

namespace psp {

// ---------------------------------------------------------------- complex
template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename C> __device__ __forceinline__ C c_add(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C c_sub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C c_mul_mi(C a) {
    return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}
template <typename C> __device__ __forceinline__ C c_zero() { return C{0, 0}; }

// Fused multiply-add written out.  The pass kernels are compiled without
// automatic contraction, so every instantiation (radix plan, tile shape,
// batched or single) rounds the same expression the same way.
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// --------------------------------------------------------------- twiddles
// Table of W_N^m = exp(-2 pi i m / N), 0 <= m < N, in FP64 for both
// tiers.  Two ways to get a butterfly's powers W^{m r}, r = 1..R-1:
// Twiddle loads the one entry W^m from the global table and forms the powers
// by a multiplication tree of depth <= 4 (a few ulp of FP64; one load instead
// of R-1, since wave-wide loads cost L1 return bandwidth per lane), in FP64
// for both tiers (an FP32 tree would add its own rounding at every level),
// rounding each power once for the FP32 tier; TableTwiddle (below) reads
// each power from a copy of the table in LDS.  The passes pick per kernel
// (passes.hpp, tw_commit).
__device__ __forceinline__ double2 cmul64(double2 a, double2 t) {
    return double2{fmadd(a.x, t.x, -(a.y * t.y)), fmadd(a.x, t.y, a.y * t.x)};
}
template <bool INV> __device__ __forceinline__ double2 cmul64_dir(double2 a, double2 t) {
    return cmul64(a, INV ? double2{t.x, -t.y} : t);
}
// p[r] = W^{m r} for r = 1..R-1 from p[1] = W^m
template <int R> __device__ __forceinline__ void twiddle_powers(double2 *p) {
    if constexpr (R > 2) p[2] = cmul64(p[1], p[1]);
    if constexpr (R > 3) p[3] = cmul64(p[2], p[1]);
    if constexpr (R > 4) {
        p[4] = cmul64(p[2], p[2]);
        p[5] = cmul64(p[4], p[1]);
        p[6] = cmul64(p[4], p[2]);
        p[7] = cmul64(p[4], p[3]);
    }
    if constexpr (R > 8) {
        p[8] = cmul64(p[4], p[4]);
#pragma unroll
        for (int k = 1; k < R - 8; ++k) p[8 + k] = cmul64(p[8], p[k]);
    }
    static_assert(R == 2 || R == 3 || R == 4 || R == 8 || R == 12 || R == 16, "radix");
}

template <typename T> struct Twiddle {
    const double2 *w;
    // v[r] *= W^{m r}, r = 1..R-1 (conjugated for the inverse transform)
    template <int R, bool INV> __device__ __forceinline__ void apply(cplx<T> *v, int m) const {
        double2 p[R];
        p[1] = w[m];
        twiddle_powers<R>(p);
#pragma unroll
        for (int r = 1; r < R; ++r) {
            if constexpr (sizeof(T) == 8) {
                v[r] = cmul64_dir<INV>(v[r], p[r]);
            } else {
                const float tx = (float)p[r].x, ty = INV ? -(float)p[r].y : (float)p[r].y;
                v[r] = float2{fmadd(v[r].x, tx, -(v[r].y * ty)), fmadd(v[r].x, ty, v[r].y * tx)};
            }
        }
    }
};

// Most passes instead read each power from a table of the roots themselves:
// at stage s a butterfly's twiddle index is m = k N/(Ns R) with k < Ns, so
// m r < N for every leg r < R and W^{m r} is an entry (the inverse
// multiplies by its conjugate; the table has the N roots W^0 .. W^{N-1}).  No
// power tree, and in FP64 each power is correctly rounded instead of a few
// ulp off.  The table is the FP64 one (FP64 tier) or its entries rounded once
// to FP32 (FP32 tier), as a copy in the workgroup's LDS or, in the persistent
// batched kernels, read from the FP64 table in global memory.  An FP32 entry
// rounded from the root equals the FP64 tree's power rounded to FP32 except
// when the root lies within a few FP64 ulp of an FP32 rounding boundary (the
// solves measured with both are bitwise equal), so FP32 passes that keep the
// trees (small workgroups) agree with the table ones.
template <typename T, int NN> struct TableTwiddle {
    const cplx<T> *t;   // NN entries, W^e for e < NN
    template <int R, bool INV> __device__ __forceinline__ void apply(cplx<T> *v, int m) const {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const cplx<T> p = t[m * r];
            const T py = INV ? -p.y : p.y;   // the inverse multiplies by the conjugate
            v[r] = cplx<T>{fmadd(v[r].x, p.x, -(v[r].y * py)), fmadd(v[r].x, py, v[r].y * p.x)};
        }
    }
};

// ------------------------------------------------------------- butterflies
template <int R, bool INV, typename C> struct DFT;

template <bool INV, typename C> struct DFT<2, INV, C> {
    __device__ __forceinline__ static void run(C *v) {
        C a = v[0], b = v[1];
        v[0] = c_add(a, b);
        v[1] = c_sub(a, b);
    }
};

template <bool INV, typename C> struct DFT<3, INV, C> {
    __device__ __forceinline__ static void run(C *v) {
        using T = decltype(v[0].x);
        const T half = T(0.5);
        const T s3 = T(0.86602540378443864676372317075293618);  // sqrt(3)/2
        C s = c_add(v[1], v[2]);
        C d = c_sub(v[1], v[2]);
        C m = C{fmadd(-half, s.x, v[0].x), fmadd(-half, s.y, v[0].y)};
        // forward: X1 = m - i s3 d, X2 = m + i s3 d
        C t = c_mul_mi<INV>(C{s3 * d.x, s3 * d.y});
        v[0] = c_add(v[0], s);
        v[1] = c_add(m, t);
        v[2] = c_sub(m, t);
    }
};

template <bool INV, typename C> struct DFT<4, INV, C> {
    __device__ __forceinline__ static void run(C *v) {
        C a = c_add(v[0], v[2]), b = c_sub(v[0], v[2]);
        C c = c_add(v[1], v[3]), d = c_mul_mi<INV>(c_sub(v[1], v[3]));
        v[0] = c_add(a, c);
        v[2] = c_sub(a, c);
        v[1] = c_add(b, d);
        v[3] = c_sub(b, d);
    }
};

template <bool INV, typename C> struct DFT<8, INV, C> {
    __device__ __forceinline__ static void run(C *v) {
        using T = decltype(v[0].x);
        const T r2 = T(0.70710678118654752440084436210484904);  // 1/sqrt(2)
        C a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = c_add(v[j], v[j + 4]);
            b[j] = c_sub(v[j], v[j + 4]);
        }
        // b_j *= W8^j (forward W8 = (1 - i)/sqrt2; inverse its conjugate)
        if (!INV) {
            b[1] = C{r2 * (b[1].x + b[1].y), r2 * (b[1].y - b[1].x)};
            b[2] = C{b[2].y, -b[2].x};
            b[3] = C{r2 * (b[3].y - b[3].x), -r2 * (b[3].x + b[3].y)};
        } else {
            b[1] = C{r2 * (b[1].x - b[1].y), r2 * (b[1].x + b[1].y)};
            b[2] = C{-b[2].y, b[2].x};
            b[3] = C{-r2 * (b[3].x + b[3].y), r2 * (b[3].x - b[3].y)};
        }
        DFT<4, INV, C>::run(a);
        DFT<4, INV, C>::run(b);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[2 * j] = a[j];
            v[2 * j + 1] = b[j];
        }
    }
};

// v *= W16^E (forward W16 = exp(-2 pi i/16); inverse its conjugate) for the
// exponents the 4 x 4 split of a length-16 DFT needs
template <int E, bool INV, typename C> __device__ __forceinline__ C mul_w16(C a) {
    using T = decltype(a.x);
    const T c1 = T(0.92387953251128675612818318939678829);   // cos(pi/8)
    const T s1 = T(0.38268343236508977172845998403039887);   // sin(pi/8)
    const T r2 = T(0.70710678118654752440084436210484904);   // 1/sqrt(2)
    T wr, wi;                                                // W16^E, forward
    if constexpr (E == 0) return a;
    else if constexpr (E == 4) return c_mul_mi<INV>(a);
    else {
        if constexpr (E == 1) { wr = c1; wi = -s1; }
        else if constexpr (E == 2) { wr = r2; wi = -r2; }
        else if constexpr (E == 3) { wr = s1; wi = -c1; }
        else if constexpr (E == 6) { wr = -r2; wi = -r2; }
        else { static_assert(E == 9, "exponent"); wr = -c1; wi = s1; }
        if (INV) wi = -wi;
        return C{fmadd(a.x, wr, -(a.y * wi)), fmadd(a.x, wi, a.y * wr)};
    }
}

// length 16 as 4 x 4: X[k1 + 4 k2] = sum_r1 W4^(r1 k2) W16^(r1 k1)
// sum_r2 W4^(r2 k1) x[r1 + 4 r2]
template <bool INV, typename C> struct DFT<16, INV, C> {
    __device__ __forceinline__ static void run(C *v) {
        C a[4][4];
#pragma unroll
        for (int r1 = 0; r1 < 4; ++r1) {
#pragma unroll
            for (int r2 = 0; r2 < 4; ++r2) a[r1][r2] = v[r1 + 4 * r2];
            DFT<4, INV, C>::run(a[r1]);            // a[r1][k1]
        }
        a[1][1] = mul_w16<1, INV>(a[1][1]);
        a[1][2] = mul_w16<2, INV>(a[1][2]);
        a[1][3] = mul_w16<3, INV>(a[1][3]);
        a[2][1] = mul_w16<2, INV>(a[2][1]);
        a[2][2] = mul_w16<4, INV>(a[2][2]);
        a[2][3] = mul_w16<6, INV>(a[2][3]);
        a[3][1] = mul_w16<3, INV>(a[3][1]);
        a[3][2] = mul_w16<6, INV>(a[3][2]);
        a[3][3] = mul_w16<9, INV>(a[3][3]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            C b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            DFT<4, INV, C>::run(b);                 // b[k2]
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
        }
    }
};

// v *= W12^E (forward W12 = exp(-2 pi i/12)) for the split of a length-12
// DFT into four 3-point DFTs (inputs 4 n1 + n2) and three 4-point DFTs
// (outputs k1 + 3 k2), with the twelfth roots of unity written out
template <int E, bool INV, typename C> __device__ __forceinline__ C mul_w12(C a) {
    using T = decltype(a.x);
    const T h3 = T(0.86602540378443864676372317075293618);   // cos(pi/6)
    T wr, wi;
    if constexpr (E == 3) return c_mul_mi<INV>(a);
    else if constexpr (E == 6) return C{-a.x, -a.y};
    else {
        if constexpr (E == 1) { wr = h3; wi = T(-0.5); }
        else if constexpr (E == 2) { wr = T(0.5); wi = -h3; }
        else { static_assert(E == 4, "exponent"); wr = T(-0.5); wi = -h3; }
        if (INV) wi = -wi;
        return C{fmadd(a.x, wr, -(a.y * wi)), fmadd(a.x, wi, a.y * wr)};
    }
}
template <bool INV, typename C> struct DFT<12, INV, C> {
    __device__ __forceinline__ static void run(C *v) {
        C a[4][3];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 3; ++n1) a[n2][n1] = v[4 * n1 + n2];
            DFT<3, INV, C>::run(a[n2]);            // a[n2][k1]
        }
        a[1][1] = mul_w12<1, INV>(a[1][1]);
        a[1][2] = mul_w12<2, INV>(a[1][2]);
        a[2][1] = mul_w12<2, INV>(a[2][1]);
        a[2][2] = mul_w12<4, INV>(a[2][2]);
        a[3][1] = mul_w12<3, INV>(a[3][1]);
        a[3][2] = mul_w12<6, INV>(a[3][2]);
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            C b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            DFT<4, INV, C>::run(b);                 // b[k2]
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 3 * k2] = b[k2];
        }
    }
};

// ------------------------------------------------------------ radix plans
// Forward radix sequence per padded length; variant PV = 0 is the default,
// PV = 1 an alternative ordering or factorisation and PV = 2 a factorisation
// with radix 16 that the autotuner may pick (where the length has them).  The first radix is even so that
// the zero-padded half of an input (and, in reverse, the cropped half of an
// output) falls on whole butterfly legs.
template <int N, int PV> struct Plan;
#define PSP_PLAN(NN, PVV, ...)                                               \
    template <> struct Plan<NN, PVV> {                                      \
        static constexpr int r[] = {__VA_ARGS__};                           \
        static constexpr int S = sizeof(r) / sizeof(int);                   \
    };
PSP_PLAN(8, 0, 8)
PSP_PLAN(12, 0, 4, 3)
PSP_PLAN(16, 0, 4, 4)
PSP_PLAN(24, 0, 8, 3)
PSP_PLAN(32, 0, 8, 4)
PSP_PLAN(48, 0, 4, 4, 3)
PSP_PLAN(64, 0, 8, 8)
PSP_PLAN(96, 0, 8, 4, 3)
PSP_PLAN(128, 0, 8, 4, 4)
PSP_PLAN(192, 0, 8, 8, 3)
PSP_PLAN(256, 0, 8, 8, 4)
PSP_PLAN(384, 0, 8, 4, 4, 3)
PSP_PLAN(512, 0, 8, 8, 8)
PSP_PLAN(768, 0, 8, 8, 4, 3)
// lengths 2^a 3^b with b >= 2: radix-3 stages (radix 12 where it saves a
// stage and keeps every thread busy)
PSP_PLAN(36, 0, 4, 3, 3)
PSP_PLAN(72, 0, 8, 3, 3)
PSP_PLAN(108, 0, 4, 3, 3, 3)
PSP_PLAN(144, 0, 8, 2, 3, 3)
PSP_PLAN(216, 0, 8, 3, 3, 3)
PSP_PLAN(288, 0, 8, 4, 3, 3)
PSP_PLAN(324, 0, 12, 3, 3, 3)
PSP_PLAN(432, 0, 12, 12, 3)
PSP_PLAN(576, 0, 12, 12, 4)
PSP_PLAN(648, 0, 8, 3, 3, 3, 3)
// alternatives
PSP_PLAN(128, 1, 4, 8, 4)
PSP_PLAN(256, 1, 4, 8, 8)
PSP_PLAN(384, 1, 12, 4, 8)
PSP_PLAN(512, 1, 8, 4, 4, 4)
PSP_PLAN(768, 1, 12, 8, 8)
// radix-16 alternatives (radix 12 for 768): one FFT stage (and LDS exchange)
// fewer where the length allows it
PSP_PLAN(128, 2, 16, 8)
PSP_PLAN(192, 2, 16, 4, 3)
PSP_PLAN(256, 2, 16, 16)
PSP_PLAN(384, 2, 16, 8, 3)
PSP_PLAN(512, 2, 16, 8, 4)
PSP_PLAN(768, 2, 8, 8, 12)
#undef PSP_PLAN

template <int N, bool INV, int PV> struct Seq {
    using P = Plan<N, PV>;
    static constexpr int S = P::S;
    __host__ __device__ static constexpr int radix(int s) { return INV ? P::r[S - 1 - s] : P::r[s]; }
    __host__ __device__ static constexpr int ns(int s) {  // product of the radices before s
        int p = 1;
        for (int i = 0; i < s; ++i) p *= radix(i);
        return p;
    }
};

// threads per column: one butterfly of the largest radix each per stage
template <int N, int PV = 0> struct MaxRadix {
    static constexpr int value() {
        int m = 0;
        for (int i = 0; i < Plan<N, PV>::S; ++i) m = Plan<N, PV>::r[i] > m ? Plan<N, PV>::r[i] : m;
        return m;
    }
};

// ---------------------------------------------------------------- engine
// Column transform engine.  TPC threads per column; thread t owns butterflies
// j = t + b*TPC (b < BPT(s)) of every stage.  LdsIdx maps (position, column)
// to an LDS element offset.
template <typename T, int N, int TPC, bool INV, int PV = 0> struct Engine {
    using C = cplx<T>;
    using Q = Seq<N, INV, PV>;
    static constexpr int S = Q::S;
    __host__ __device__ static constexpr int R(int s) { return Q::radix(s); }
    __host__ __device__ static constexpr int NS(int s) { return Q::ns(s); }
    __host__ __device__ static constexpr int BPT(int s) { return (N / R(s) + TPC - 1) / TPC; }
    static constexpr int maxv() {
        int m = 0;
        for (int s = 0; s < S; ++s) m = BPT(s) * R(s) > m ? BPT(s) * R(s) : m;
        return m;
    }
    static constexpr int V = maxv();

    // butterflies of stage s on registers (twiddle, then radix-R DFT)
    template <int s, typename TW>
    __device__ __forceinline__ static void compute(C *v, int t, const TW &tw) {
        constexpr int r_ = R(s), ns_ = NS(s), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(s); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
                C *w = v + b * r_;
                if (ns_ > 1) {
                    const int k = j % ns_;
                    constexpr int stride = N / (ns_ * r_);
                    tw.template apply<r_, INV>(w, k * stride);
                }
                DFT<r_, INV, C>::run(w);
            }
        }
    }

    // output position of leg r of butterfly j at stage s
    template <int s> __device__ __forceinline__ static int out_pos(int j, int r) {
        constexpr int r_ = R(s), ns_ = NS(s);
        return (j / ns_) * ns_ * r_ + (j % ns_) + r * ns_;
    }
    // input position of leg r of butterfly j at stage s
    template <int s> __device__ __forceinline__ static int in_pos(int j, int r) {
        return j + r * (N / R(s));
    }

    template <int s, typename Idx>
    __device__ __forceinline__ static void store_lds(const C *v, C *lds, int t, Idx idx) {
        constexpr int r_ = R(s), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(s); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
#pragma unroll
                for (int r = 0; r < r_; ++r) lds[idx(out_pos<s>(j, r))] = v[b * r_ + r];
            }
        }
    }
    template <int s, typename Idx>
    __device__ __forceinline__ static void load_lds(C *v, const C *lds, int t, Idx idx) {
        constexpr int r_ = R(s), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(s); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
#pragma unroll
                for (int r = 0; r < r_; ++r) v[b * r_ + r] = lds[idx(in_pos<s>(j, r))];
            }
        }
    }

    // half-buffer exchange: phase ph moves the values whose position lies in
    // [ph N/2, (ph+1) N/2) through an LDS buffer of N/2 positions
    template <int s, typename Idx>
    __device__ __forceinline__ static void store_half(const C *v, C *lds, int t, Idx idx, int ph) {
        constexpr int r_ = R(s), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(s); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
#pragma unroll
                for (int r = 0; r < r_; ++r) {
                    const int pos = out_pos<s>(j, r);
                    if ((pos >= N / 2) == (ph == 1)) lds[idx(pos - ph * (N / 2))] = v[b * r_ + r];
                }
            }
        }
    }
    template <int s, typename Idx>
    __device__ __forceinline__ static void load_half(C *v, const C *lds, int t, Idx idx, int ph) {
        constexpr int r_ = R(s), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(s); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
#pragma unroll
                for (int r = 0; r < r_; ++r) {
                    const int pos = in_pos<s>(j, r);
                    // for even radices the upper half is exactly legs r >= R/2
                    const bool upper = (r_ % 2 == 0) ? (r >= r_ / 2) : (pos >= N / 2);
                    if (upper == (ph == 1)) v[b * r_ + r] = lds[idx(pos - ph * (N / 2))];
                }
            }
        }
    }

    // copy the lower-half inputs of stage s from lo into v
    template <int s>
    __device__ __forceinline__ static void merge_lower(C *v, const C *lo, int t) {
        constexpr int r_ = R(s), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(s); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
#pragma unroll
                for (int r = 0; r < r_; ++r) {
                    const int pos = in_pos<s>(j, r);
                    const bool upper = (r_ % 2 == 0) ? (r >= r_ / 2) : (pos >= N / 2);
                    if (!upper) v[b * r_ + r] = lo[b * r_ + r];
                }
            }
        }
    }

    // stages [s, S) given stage-s inputs in registers; on return registers
    // hold the last stage's outputs at positions j + r N/R(S-1).  SPLIT: each
    // exchange goes through an LDS buffer of N/2 positions in two phases.
    template <int s, bool SPLIT = false, typename Idx, typename TW>
    __device__ __forceinline__ static void run_from(C *v, C *lds, int t, Idx idx, const TW &tw) {
        compute<s>(v, t, tw);
        if constexpr (s + 1 < S) {
            if constexpr (SPLIT) {
                // the phase-0 inputs of stage s+1 must not overwrite stage-s
                // outputs still waiting for phase 1: stage them in lo[]
                C lo[V];
                store_half<s>(v, lds, t, idx, 0);
                __syncthreads();
                load_half<s + 1>(lo, lds, t, idx, 0);
                __syncthreads();
                store_half<s>(v, lds, t, idx, 1);
                __syncthreads();
                load_half<s + 1>(v, lds, t, idx, 1);
                __syncthreads();
                merge_lower<s + 1>(v, lo, t);
            } else {
                store_lds<s>(v, lds, t, idx);
                __syncthreads();
                load_lds<s + 1>(v, lds, t, idx);
                __syncthreads();
            }
            run_from<s + 1, SPLIT>(v, lds, t, idx, tw);
        }
    }

    // stages [s, S) with every exchange in two phases by column half: the
    // threads of the first half of the workgroup's columns store and load
    // through an LDS buffer of half the columns, then those of the second
    // half (idx addresses the half buffer).  Each thread stores all its
    // values before loading, so no value needs a staging register.
    template <int s, typename Idx, typename TW>
    __device__ __forceinline__ static void run_from_cols(C *v, C *lds, int t, Idx idx, const TW &tw,
                                                         bool first_half) {
        compute<s>(v, t, tw);
        if constexpr (s + 1 < S) {
            if (first_half) store_lds<s>(v, lds, t, idx);
            __syncthreads();
            if (first_half) load_lds<s + 1>(v, lds, t, idx);
            __syncthreads();
            if (!first_half) store_lds<s>(v, lds, t, idx);
            __syncthreads();
            if (!first_half) load_lds<s + 1>(v, lds, t, idx);
            __syncthreads();
            run_from_cols<s + 1>(v, lds, t, idx, tw, first_half);
        }
    }

    // visit the final outputs: f(position, leg r, value&); legs r < R/2 of
    // the last stage are exactly the positions below N/2
    template <typename F>
    __device__ __forceinline__ static void for_outputs(C *v, int t, F f) {
        constexpr int s = S - 1, r_ = R(s), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(s); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
#pragma unroll
                for (int r = 0; r < r_; ++r) f(j + r * nb, r, v[b * r_ + r]);
            }
        }
    }
    // fill the first-stage inputs: v = g(position, leg r); legs r < R/2 of
    // the first stage are exactly the positions below N/2
    template <typename G>
    __device__ __forceinline__ static void for_inputs(C *v, int t, G g) {
        constexpr int r_ = R(0), nb = N / r_;
#pragma unroll
        for (int b = 0; b < BPT(0); ++b) {
            const int j = t + b * TPC;
            if ((nb % TPC == 0) || j < nb) {
#pragma unroll
                for (int r = 0; r < r_; ++r) v[b * r_ + r] = g(j + r * nb, r);
            }
        }
    }
};

}  // namespace psp
