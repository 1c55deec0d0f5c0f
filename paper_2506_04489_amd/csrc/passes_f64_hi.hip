// passes_f64_hi.hip - the FP64 instantiation of the solve passes for
// padded lengths 256 to 768.
#include "passes.hpp"

namespace psp {

hipError_t passes_f64_hi PSP_PASSES_SIGNATURE {
    switch (N) {
        PSP_CASE(double, 256)
        PSP_CASE(double, 384)
        PSP_CASE(double, 512)
        PSP_CASE(double, 768)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psp
