// batch.cpp -- hlb_cp_mm_batch: many CP-MMs of uneven shapes over shared primes.
#include <hip/hip_runtime.h>

#include "../../include/hlb.h"
#include "host.hpp"

namespace hlb {
void batch_release() {}
}  // namespace hlb

extern "C" hlb_status hlb_cp_mm_batch(const hlb_cpmm_problem *probs, int count, const uint64_t *primes, int L,
                                      int form, void *stream) {
    if (count < 0 || (count > 0 && !probs)) return HLB_EINVAL;
    for (int i = 0; i < count; ++i) {
        const hlb_cpmm_problem &p = probs[i];
        hlb_status st = hlb_cp_mm(p.m, p.k, p.nA, p.nB, p.P, p.ldp, p.p_absmax, p.A, p.B, primes, L, p.PA, p.PB,
                                  form, stream);
        if (st != HLB_OK) return st;
    }
    return HLB_OK;
}
