// passes_f64_lo.hip - the FP64 instantiation of the solve passes for
// padded lengths 8 to 192.
#include "passes.hpp"

namespace psp {

hipError_t passes_f64_lo PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(double, 8)
        PSP_CASE(double, 12)
        PSP_CASE(double, 16)
        PSP_CASE(double, 24)
        PSP_CASE(double, 32)
        PSP_CASE(double, 48)
        PSP_CASE(double, 64)
        PSP_CASE(double, 96)
        PSP_CASE(double, 128)
        PSP_CASE(double, 192)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
