// passes_f64.hip - the FP64 instantiation of the solve passes.
#include "passes.hpp"

namespace psp {

hipError_t passes_f64(int N, const Job &one, const Job *table, int count, int P, int chunk_tiles, int i1_group,
                      const Shape &sh, bool full, const void *tw_hi, const void *tw_lo, hipEvent_t *ev, int *ev_pass,
                      int nev, hipStream_t st) {
    return passes_dispatch<double>(N, one, table, count, P, chunk_tiles, i1_group, sh, full, tw_hi, tw_lo, ev,
                                   ev_pass, nev, st);
}

}  // namespace psp
