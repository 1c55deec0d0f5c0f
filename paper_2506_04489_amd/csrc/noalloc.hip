// noalloc.hip - psp_solve_noalloc: the solve of psp_solve with its two
// intermediates (X and A) placed in a fixed file-scope device array instead
// of a library allocation, for callers that cannot allocate device memory.
//
// The array `scratch` is a module global: every GPU the library runs on holds
// its own copy, kNoAllocBytes large, until the process ends.  Host code never
// uses the name `scratch` as an address (on the host it is only a stand-in
// for the symbol); the device address of each GPU's copy is looked up once
// per device with hipGetSymbolAddress on the first call made with that device
// current, and that pointer is what the kernels receive.
#include <cstring>

#include "host_common.hpp"

namespace psp {

constexpr size_t kNoAllocBytes = (size_t)128 << 20;   // the array's size: 128 MiB
constexpr int kNoAllocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kNoAllocDevices];   // device address of each GPU's copy

// the current device's copy of `scratch` (looked up once per device)
static psp_status noalloc_scratch(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kNoAllocDevices) return fail(PSP_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(PSP_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = (unsigned char *)g_noalloc_ptr[dev];
    return PSP_OK;
}

}  // namespace psp

using namespace psp;

extern "C" {

psp_status psp_solve_noalloc(const psp_plan *p, const void *rho_dev, void *u_dev, void *stream) {
    return guarded([&]() -> psp_status {
        if (!p || !rho_dev || !u_dev) return fail(PSP_EINVAL, "NULL argument");
        if (!p->precomputed) return fail(PSP_ESTATE, "psp_solve_noalloc before psp_kernel_precompute");
        if (rho_dev == u_dev) return fail(PSP_EINVAL, "rho and u must not alias");
        int dev = -1;
        const hipError_t ge = hipGetDevice(&dev);
        if (ge != hipSuccess) return hip_fail(ge, "hipGetDevice");
        if (dev != p->device)
            return fail(PSP_EINVAL, "plan was precomputed on device %d, current is %d", p->device, dev);
        // the same two intermediates psp_solve allocates, back to back
        const bool f32 = p->dtype == PSP_F32;
        const size_t c = f32 ? 8 : 16;
        size_t x_bytes, a_bytes;
        if (p->grid) {
            const Dims d{p->ns[0], p->ns[1], p->ns[2]};
            x_bytes = c * (size_t)pitch_for(d.n3) * d.n1 * d.n2;
            a_bytes = c * a_plane(d.n1, d.n2, chunk_pitch(d.n3, f32, 0), (int)c) * d.n1;
        } else {
            const int n = p->n;
            x_bytes = c * (size_t)pitch_for(n) * x_slabs(n, f32, p->chunk_tiles, p->i1_group) * n;
            a_bytes = c * a_plane(n, n, chunk_pitch(n, f32, p->chunk_tiles), (int)c) * n;
        }
        const size_t a_off = (x_bytes + 255) & ~(size_t)255;
        if (a_off + a_bytes > kNoAllocBytes)
            return fail(PSP_ENOMEM, "the solve needs %zu bytes of intermediates, more than the %zu bytes of the "
                                    "static scratch array",
                        a_off + a_bytes, kNoAllocBytes);
        unsigned char *base = nullptr;
        psp_status rs = noalloc_scratch(dev, &base);
        if (rs != PSP_OK) return rs;
        Workspace w;
        w.X = base;
        w.A = base + a_off;
        w.bytes = a_off + a_bytes;
        // no profiling events and no guard bands: the passes, nothing else
        SolveArgs a = solve_args(p, w, rho_dev, u_dev);
        const hipError_t e = launch_solve(a, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "solve launch");
        return PSP_OK;
    });
}

}  // extern "C"
