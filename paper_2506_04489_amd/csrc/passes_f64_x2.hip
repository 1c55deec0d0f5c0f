// passes_f64_x2.hip - the F64 instantiation of the solve passes for the
// padded lengths 288 to 648 with a factor 9.
#include "passes.hpp"

namespace psp {

hipError_t passes_f64_x2 PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(double, 288)
        PSP_CASE(double, 324)
        PSP_CASE(double, 432)
        PSP_CASE(double, 576)
        PSP_CASE(double, 648)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
