// passes_f64_x1.hip - the F64 instantiation of the solve passes for the
// padded lengths 36 to 216 with a factor 9.
#include "passes.hpp"

namespace psp {

hipError_t passes_f64_x1 PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(double, 36)
        PSP_CASE(double, 72)
        PSP_CASE(double, 108)
        PSP_CASE(double, 144)
        PSP_CASE(double, 216)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
