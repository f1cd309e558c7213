// gemm_i8_trunc.hip -- INT8 limb GEMM that keeps only the high-order digit products.
//
// Strategy 2 of Section 6.1 truncates the decomposition of Eq decomp to its largest terms;
// the paper notes that compromises between Strategies 1 and 2 come from varying how many
// terms are kept.  In the INT8 form that means skipping the digit products P_i X_j of the
// lowest shifts i + j < DROP: the kernel then returns (V - D) mod q, where V is the exact
// product and D = sum over the skipped pairs of c_{ij} 256^(i+j) is an integer with
// |D| <= k 2^14 sum_{s < DROP} pairs(s) 256^s.  Used for the b-part of a CP-MM, whose error
// reaches the decrypted message unamplified.
#include "common.hpp"
#include "i8_tile.hpp"
#include "launch.hpp"

namespace hlb {

template <int DROP>
static hipError_t launch_drop(int dp, int dx, int cls, const GemmArgs &a, hipStream_t s) {
    // the planner keeps truncated products to K ranges that need no fold
    if (a.kfold < a.kblocks) return hipErrorInvalidValue;
    if (dp == 3 && dx == 7)
        return cls == 1 ? launch_gemm_t<Class1<3, 7, DROP>, false>(a, s) : launch_gemm_t<Class0<3, 7, DROP>, false>(a, s);
    if (dp == 3 && dx == 6)
        return cls == 1 ? launch_gemm_t<Class1<3, 6, DROP>, false>(a, s) : launch_gemm_t<Class0<3, 6, DROP>, false>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_gemm_i8_trunc(int dp, int dx, int cls, int drop, const GemmArgs &a, hipStream_t s) {
    switch (drop) {
        case 1: return launch_drop<1>(dp, dx, cls, a, s);
        case 2: return launch_drop<2>(dp, dx, cls, a, s);
        case 3: return launch_drop<3>(dp, dx, cls, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hlb
