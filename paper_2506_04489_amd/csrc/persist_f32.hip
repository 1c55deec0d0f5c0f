// persist_f32.hip - FP32-tier instantiation of the persistent batched passes.
#define PB_LDS_ELEM float2
#include "persist.hpp"

namespace psp {

const void *persist_kernel_f32(int pass) {
    switch (pass) {
        case 0: return (const void *)k_persist<float, 0>;
        case 1: return (const void *)k_persist<float, 1>;
        case 2: return (const void *)k_persist<float, 2>;
        case 3: return (const void *)k_persist<float, 3>;
        default: return (const void *)k_persist<float, 4>;
    }
}

hipError_t persist_launch_f32(PBatch *d_hdr, const int *total, const int *grid, hipStream_t st) {
    (void)total;
    hipLaunchKernelGGL((k_persist<float, 0>), dim3(grid[0]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<float, 1>), dim3(grid[1]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<float, 2>), dim3(grid[2]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<float, 3>), dim3(grid[3]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_persist<float, 4>), dim3(grid[4]), dim3(PB_THREADS), 0, st, d_hdr);
    return hipGetLastError();
}

hipError_t flat_launch_f32(PBatch *d_hdr, const int *total, hipStream_t st) {
    hipLaunchKernelGGL((k_flat<float, 0>), dim3(total[0]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<float, 1>), dim3(total[1]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<float, 2>), dim3(total[2]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<float, 3>), dim3(total[3]), dim3(PB_THREADS), 0, st, d_hdr);
    hipLaunchKernelGGL((k_flat<float, 4>), dim3(total[4]), dim3(PB_THREADS), 0, st, d_hdr);
    return hipGetLastError();
}

}  // namespace psp
