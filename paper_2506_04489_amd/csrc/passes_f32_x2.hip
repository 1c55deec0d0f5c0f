// passes_f32_x2.hip - the F32 instantiation of the solve passes for the
// padded lengths 288 to 648 with a factor 9.
#include "passes.hpp"

namespace psp {

hipError_t passes_f32_x2 PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(float, 288)
        PSP_CASE(float, 324)
        PSP_CASE(float, 432)
        PSP_CASE(float, 576)
        PSP_CASE(float, 648)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
