// persist_f64.hip - FP64 instantiation of the persistent batched passes,
// the counter reset and the launcher shared by both precisions.
#include <mutex>

#include "persist.hpp"

namespace psp {

__global__ void k_pb_reset(PBatch *bt) {
    if (threadIdx.x < kPasses) bt->counter[threadIdx.x] = 0;
}

template <int N, int PV> static int tpc_of() { return PBCfg<N, PV>::TPC; }

int persist_tpc(int N, int pv) {
    switch (N) {
        case 8: return tpc_of<8, 0>();
        case 12: return tpc_of<12, 0>();
        case 16: return tpc_of<16, 0>();
        case 24: return tpc_of<24, 0>();
        case 32: return tpc_of<32, 0>();
        case 48: return tpc_of<48, 0>();
        case 64: return tpc_of<64, 0>();
        case 96: return tpc_of<96, 0>();
        case 128: return pv ? tpc_of<128, 1>() : tpc_of<128, 0>();
        case 192: return tpc_of<192, 0>();
        case 256: return pv ? tpc_of<256, 1>() : tpc_of<256, 0>();
        default: return 0;
    }
}

// resident workgroups of each persistent kernel on the current device
struct PersistGrid {
    int dev = -1;
    int blocks[2][kPasses] = {};
};

hipError_t persist_launch_f32(PBatch *d_hdr, const int *total, const int *grid, hipStream_t st);
const void *persist_kernel_f32(int pass);

static const void *kernel_f64(int pass) {
    switch (pass) {
        case 0: return (const void *)k_persist<double, 0>;
        case 1: return (const void *)k_persist<double, 1>;
        case 2: return (const void *)k_persist<double, 2>;
        case 3: return (const void *)k_persist<double, 3>;
        default: return (const void *)k_persist<double, 4>;
    }
}

static hipError_t grids(PersistGrid *g) {
    static std::mutex mu;
    static PersistGrid cache[16];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 16) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (cache[dev].dev != dev) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        for (int t = 0; t < 2; ++t)
            for (int p = 0; p < kPasses; ++p) {
                int per = 0;
                const void *k = t ? persist_kernel_f32(p) : kernel_f64(p);
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, PB_THREADS, 0);
                if (e != hipSuccess) return e;
                cache[dev].blocks[t][p] = (per > 0 ? per : 1) * cus;
            }
        cache[dev].dev = dev;
    }
    *g = cache[dev];
    return hipSuccess;
}

hipError_t persist_prepare() {
    PersistGrid g;
    return grids(&g);
}

hipError_t flat_launch_f32(PBatch *d_hdr, const int *total, hipStream_t st);

hipError_t flat_launch(bool f32, PBatch *d_hdr, const int *total, hipStream_t st) {
    if (f32) return flat_launch_f32(d_hdr, total, st);
    hipLaunchKernelGGL((k_flat<double, 0>), dim3(total[0]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<double, 1>), dim3(total[1]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<double, 2>), dim3(total[2]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<double, 3>), dim3(total[3]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<double, 4>), dim3(total[4]), dim3(PB_THREADS), 0, st, d_hdr);
    return hipGetLastError();
}

hipError_t persist_launch(bool f32, PBatch *d_hdr, const int *total, bool reset, hipStream_t st) {
    PersistGrid g;
    hipError_t e = grids(&g);
    if (e != hipSuccess) return e;
    if (reset) {
        hipLaunchKernelGGL(k_pb_reset, dim3(1), dim3(64), 0, st, d_hdr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int grid[kPasses];
    for (int p = 0; p < kPasses; ++p) grid[p] = std::max(1, std::min(total[p], g.blocks[f32 ? 1 : 0][p]));
    if (f32) return persist_launch_f32(d_hdr, total, grid, st);
    hipLaunchKernelGGL((k_persist<double, 0>), dim3(grid[0]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<double, 1>), dim3(grid[1]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<double, 2>), dim3(grid[2]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<double, 3>), dim3(grid[3]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<double, 4>), dim3(grid[4]), dim3(PB_THREADS), 0, st, d_hdr);
    return hipGetLastError();
}

}  // namespace psp
