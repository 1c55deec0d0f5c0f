// passes_f32_x1.hip - the F32 instantiation of the solve passes for the
// padded lengths 36 to 216 with a factor 9.
#include "passes.hpp"

namespace psp {

hipError_t passes_f32_x1 PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(float, 36)
        PSP_CASE(float, 72)
        PSP_CASE(float, 108)
        PSP_CASE(float, 144)
        PSP_CASE(float, 216)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
