// passes_f32_hi.hip - the FP32-tier instantiation of the solve passes (FP32
// data and arithmetic, split FP32 twiddles, FP64 multiplier), padded lengths
// 256 to 768.
#include "passes.hpp"

namespace psp {

hipError_t passes_f32_hi PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(float, 256)
        PSP_CASE(float, 384)
        PSP_CASE(float, 512)
        PSP_CASE(float, 768)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
