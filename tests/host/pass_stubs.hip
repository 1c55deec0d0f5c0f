// Stand-ins for the FFT pass instantiations and the persistent batch kernels
// in the sanitized host build of libpsp (tests/host/sanitized.py): that build
// exercises host logic only, never launches a pass, and leaves out the
// translation units whose device code takes minutes to compile.  Every stand-in
// reports failure, so a path that did reach a launch would return an error.
#include <hip/hip_runtime.h>

#include "../../paper_2506_04489_amd/csrc/kernels.h"

namespace psp {

#define PSP_STUB_PASSES(name)                                                                               \
    hipError_t name(int, const Job &, const Job *, int, int, int, int, const Shape &, bool, const void *,  \
                    hipEvent_t *, int *, int, const Dims &, int, hipStream_t) {                            \
        return hipErrorInvalidValue;                                                                        \
    }
PSP_STUB_PASSES(passes_f64_lo)
PSP_STUB_PASSES(passes_f64_hi)
PSP_STUB_PASSES(passes_f64_x1)
PSP_STUB_PASSES(passes_f64_x2)
PSP_STUB_PASSES(passes_f32_lo)
PSP_STUB_PASSES(passes_f32_hi)
PSP_STUB_PASSES(passes_f32_x1)
PSP_STUB_PASSES(passes_f32_x2)
#undef PSP_STUB_PASSES

int persist_tpc(int, int) { return 0; }
hipError_t persist_prepare() { return hipErrorInvalidValue; }
hipError_t persist_launch(bool, PBatch *, const int *, bool, hipStream_t) { return hipErrorInvalidValue; }
hipError_t flat_launch(bool, PBatch *, const int *, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace psp
