// kernels.h - host-side launch interface of the device passes (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace psp {

// One solve's device pointers as the pass kernels see them.
struct Job {
    const void *rho = nullptr;
    void *u = nullptr;
    void *X = nullptr;           // n*n*P complex
    void *A = nullptr;           // chunk buffer
    const double *mult = nullptr;
    void *A2 = nullptr;          // uncropped variant only
    void *Y2 = nullptr;          // uncropped variant only
};

// Launch shape of the five passes H1..H5 (index p = 0..4): the autotuner's
// search space.
//   plan[p]: radix plan of the pass (0: default, 1: an alternative ordering,
//            2: a radix-16 (radix-12 for 768) factorisation, where the
//            padded length has them;
//            a different rounding, same accuracy class)
//   tile[p]: H1/H5 (p = 0, 4): workgroup size, 0: 256 threads, 1: 128, 2: 512,
//            3: 64 (one line per workgroup where a line takes 64 threads),
//            4-7: 0-3 with nontemporal stores (H1 of X, H5 of u);
//            H2-H4 (p = 1..3): 0: one 128-byte row tile of k3 columns per
//            workgroup (8 FP64 / 16 FP32 columns), 1: half of one, 2: one
//            tile with exchanges through half-size LDS buffers by position
//            half, 3: one tile with half the threads per column (two
//            butterflies each), 4: 2 and 3, 5: one tile with exchanges
//            through half-size LDS buffers by column half, 6: 5 and 3;
//            also 7-13: 0-6 with nontemporal accesses (H2 its stores of A,
//            H3 its stores of A, H4 its loads of A and stores of X); H3
//            (p = 2) also 14-20: 0-6 with nontemporal loads and stores
// A tile choice only changes which workgroup transforms which column, how
// values move between stages and the cache policy of the accesses, so
// results are bitwise the same under every tile choice.
constexpr int kPasses = 5;
constexpr int kTileChoices[kPasses] = {8, 14, 21, 14, 8};
constexpr int kMaxTiles = 21;     // the largest of kTileChoices
constexpr int kMaxPlans = 3;      // radix plans 0..2
// points along i1, i2, i3 (the slowest to the contiguous axis of rho)
struct Dims {
    int n1, n2, n3;
};

// i1 pitch, in elements of `elem` bytes, of the padded intermediate A of n1
// planes whose 2 n2 rows k2 hold `pa` columns (pa * elem a multiple of 128
// bytes).  The fused i1 pass reads each column at this stride; at a multiple
// of 4 KB those reads fall on too few HBM channels (measured: the pass's
// access pattern at n = 256 streams 10% faster at 15 mod 32 lines of 128
// bytes than at 0 mod 32).  So a buffer larger than 128 MiB gets its pitch
// rounded up to 15 mod 32 lines; a smaller one is mostly served by the
// last-level cache and keeps 2 n2 pa (padding measured no faster there).
__host__ __device__ constexpr size_t a_plane(int n1, int n2, int pa, int elem) {
    const size_t lines = (size_t)2 * n2 * pa * elem / 128;
    if (lines * 128 * (size_t)n1 <= ((size_t)128 << 20)) return lines * 128 / elem;
    return (lines + (47 - lines % 32) % 32) * 128 / elem;
}

struct Shape {
    int plan[kPasses] = {0, 0, 0, 0, 0};
    int tile[kPasses] = {0, 0, 0, 0, 0};
    bool operator==(const Shape &o) const {
        for (int p = 0; p < kPasses; ++p)
            if (plan[p] != o.plan[p] || tile[p] != o.tile[p]) return false;
        return true;
    }
    bool operator<(const Shape &o) const {
        for (int p = 0; p < kPasses; ++p) {
            if (plan[p] != o.plan[p]) return plan[p] < o.plan[p];
            if (tile[p] != o.tile[p]) return tile[p] < o.tile[p];
        }
        return false;
    }
};
// radix plans of a padded length: 0 the default; 1 an alternative ordering or
// factorisation (2n in {128, 256, 384, 512, 768}); 2 a radix-16 factorisation (2n
// in {128, 192, 256, 384, 512}) or for 768 one with radix 12
constexpr bool alt_plan_exists(int N) { return N == 128 || N == 256 || N == 384 || N == 512 || N == 768; }
constexpr bool r16_plan_exists(int N) { return N == 128 || N == 192 || N == 256 || N == 384 || N == 512 || N == 768; }
constexpr bool plan_exists(int N, int pv) {
    return pv == 0 || (pv == 1 && alt_plan_exists(N)) || (pv == 2 && r16_plan_exists(N));
}
inline bool shape_valid(int n, const Shape &s) {
    for (int p = 0; p < kPasses; ++p) {
        if (!plan_exists(2 * n, s.plan[p])) return false;
        if (s.tile[p] < 0 || s.tile[p] >= kTileChoices[p]) return false;
    }
    return true;
}

// ------------------------------------------------ persistent batched passes
constexpr int PB_THREADS = 384;   // workgroup size: divisible by every threads-per-column count
constexpr int PB_MAX_N = 256;     // largest padded length on the persistent path

// One solve of a persistent batch (device table entry).
struct PJob {
    const void *rho;
    void *u;
    void *X;                 // n*n*P complex
    void *A;                 // n planes of `plane` complex, rows of pa
    const double *mult;      // blocked multiplier octant
    const void *tw64;       // twiddles double2[N], both tiers
    int N;                   // padded length
    int P;                   // k3 pitch of X
    int pa;                  // k3 pitch of A
    int pv[kPasses];         // radix plan of each pass
    long long plane;         // i1 pitch of A (a_plane)
};

// Batch header in device memory.  counter[p] must be zero when pass p
// starts; start[p * (njobs + 1) + j] is the first item of job j in pass p
// (start[p * (njobs + 1) + njobs] = total[p]).
struct PBatch {
    int counter[kPasses];
    int total[kPasses];
    int njobs;
    int pad_;
    const PJob *jobs;
    const int *start;
};

// threads per column (strided passes) or per line (line passes) of the
// persistent kernels for padded length N and radix plan pv
int persist_tpc(int N, int pv);
// occupancy queries of the persistent kernels, cached per device (call once
// outside graph capture)
hipError_t persist_prepare();
// the five persistent passes over the batch whose header is at d_hdr;
// reset: clear the counters first (a kernel, so graphs may capture it)
hipError_t persist_launch(bool f32, PBatch *d_hdr, const int *total, bool reset, hipStream_t st);
// the same passes with one workgroup per item (grids of total[p] workgroups)
hipError_t flat_launch(bool f32, PBatch *d_hdr, const int *total, hipStream_t st);

// One solve's buffers (device pointers) and sizes.
struct SolveArgs {
    int n = 0;          // points per axis; padded length N = 2n
    int P = 0;          // pitch of the half-spectrum axis, round_up(n+1, 16)
    bool f32 = false;   // FP32 tier (data and FFT in FP32, multiplier FP64)
    bool full = false;  // uncropped (2n)^3 output (test hook)
    const void *rho = nullptr;
    void *u = nullptr;
    void *X = nullptr;   // n*n*P complex
    void *A = nullptr;   // chunk buffer: n*N*(chunk_tiles*W) complex
    int chunk_tiles = 0; // k3 tiles per H2-H4 chunk (0: all tiles in one chunk)
    int i1_group = 0;    // i1 slabs per H1-H2 / H4-H5 group (0: all; X then holds one group)
    Shape shape;         // launch shape (ignored by the uncropped variant)
    void *A2 = nullptr;  // N*N*P complex, full variant only
    void *Y2 = nullptr;  // N*N*P complex, full variant only
    const double *mult = nullptr;   // blocked multiplier octant
    const void *tw64 = nullptr;    // twiddles double2[N], both tiers
    hipEvent_t *ev = nullptr;       // optional profiling events, one before each launch and one after
    int *ev_pass = nullptr;         // host array: pass (0..4) of each launch, -1 for the last event
    int nev = 0;
    // unequal point counts per axis (ns[0] == 0: all n): each pass runs at
    // the padded length of its axis with that axis's twiddles tw_axis[]; no
    // chunking, grouping, uncropped output or profiling events
    int ns[3] = {0, 0, 0};
    const void *tw_axis[3] = {nullptr, nullptr, nullptr};
};

hipError_t launch_solve(const SolveArgs &s, hipStream_t st);

// `count` solves of the same n and tier in one launch per pass; `table_dev`
// is a device array of `count` jobs, each with a workspace of one chunk
// holding all tiles (chunk_tiles = 0)
hipError_t launch_group(int n, bool f32, const Shape &shape, const Job *table_dev, int count, const void *tw64,
                        hipStream_t st);

// k3 columns per 128-byte row tile of the padded intermediates (8 FP64, 16 FP32)
inline int strided_width(bool f32) { return f32 ? 16 : 8; }

// the kernel-spectrum multiplier octant (FP64 MFMA contraction)
// S2 inputs: the 1D tables of each axis (R x (n+1) each; the same pointers
// for every axis of a cubic box) and the epilogue's spectral-Laplacian
// weights w_p = (2 pi / L_p)^2 and scale -1/(N1 N2 N3)
struct SpecTables {
    const double *J0[3];
    const double *J2[3];
    int n[3];   // points per axis: tables of axis p have n[p] + 1 columns
};
struct SpecScale {
    double w[3];
    double scale;
};
hipError_t launch_spectrum(const SpecTables &tb, const double *omega, int R, int P, const SpecScale &sc,
                           double *mult, hipStream_t st);

// kernel launches of one solve (its profiling events are one more)
int solve_launches(int n, bool f32, int chunk_tiles, int i1_group);

// supported padded lengths: every 2^a 3^b from 8 to 768 whose half n is even
inline bool supported_length(int N) {
    switch (N) {
        case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
        case 128: case 192: case 256: case 384: case 512: case 768: return true;
        case 36: case 72: case 108: case 144: case 216: case 288: case 324: case 432: case 576: case 648:
            return true;
        default: return false;
    }
}
// lengths with a factor 9 (two or more radix-3 stages): instantiated in the
// passes_{f64,f32}_x*.hip files
inline bool nine_length(int N) { return N % 9 == 0; }

}  // namespace psp
