// passes_f32_lo.hip - the FP32-tier instantiation of the solve passes (FP32
// data and arithmetic, split FP32 twiddles, FP64 multiplier), padded lengths
// 8 to 192.
#include "passes.hpp"

namespace psp {

hipError_t passes_f32_lo PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(float, 8)
        PSP_CASE(float, 12)
        PSP_CASE(float, 16)
        PSP_CASE(float, 24)
        PSP_CASE(float, 32)
        PSP_CASE(float, 48)
        PSP_CASE(float, 64)
        PSP_CASE(float, 96)
        PSP_CASE(float, 128)
        PSP_CASE(float, 192)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
