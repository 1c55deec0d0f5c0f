// batched.hip - many independent solves on one stream.
#include "kernels.h"

namespace psp {

hipError_t launch_batch(int count, const SolveArgs *args, hipStream_t st) {
    for (int i = 0; i < count; ++i) {
        hipError_t e = launch_solve(args[i], st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace psp
