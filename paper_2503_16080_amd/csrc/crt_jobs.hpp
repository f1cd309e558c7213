// crt_jobs.hpp -- residue arithmetic and job structures of the multimodular (CRT) form's
// splits and recombination (crt.hip) and of its batch GEMM (crt_gemm_batch.hip): the int8
// residue of a value modulo each small modulus, the recombination arguments of an output
// matrix, the job tables that let one launch split many operands or recombine many output
// matrices, and the host-resolved tiles of a batch.
#pragma once

#include <stdint.h>

#include "common.hpp"
#include "crt.hpp"

namespace hlb {

// A signed integer |s| < 2^52, held as the exact double sd and its low word lo.
struct CrtValue {
    double sd;
    uint32_t lo;
};
__device__ __forceinline__ CrtValue crt_value(int64_t s) {
    const double hi = (double)(int32_t)(s >> 32);
    return {__builtin_fma(hi, 4294967296.0, (double)(uint32_t)s), (uint32_t)s};
}

// A word whose low byte is the int8 residue of s modulo p (the balanced residue; for p = 256
// the byte of s itself, where +128 and -128 coincide modulo 256).
//  * t = the nearest integer to s / p: s (1/p) + 1.5 2^52 lies in [2^52, 2^53), where doubles
//    are spaced by 1, so one fused multiply-add rounds it to 1.5 2^52 + t, whose low word is
//    t mod 2^32.  The double 1/p is within 2^-53 relative of 1/p, so s (1/p) is within
//    |s| 2^-53 / p < 1 / (2p) of s / p, while for odd p s / p lies at least 1 / (2p) from any
//    half-integer: the rounding is that of s / p itself.  For p = 256, 1/p is exact.
//  * s - t p, of magnitude at most p / 2, is then formed modulo 2^24 by one 24-bit
//    multiply-add with 2^24 - p, and its low byte is the residue.
template <int P>
__device__ __forceinline__ uint32_t crt_residue_word(const CrtValue &v) {
    if constexpr (P == 256) {
        return v.lo;
    } else {
        const double td = __builtin_fma(v.sd, 1.0 / (double)P, 6755399441055744.0);
        const uint32_t t = (uint32_t)__double2loint(td);
        return __umul24(t, (1u << 24) - (uint32_t)P) + v.lo;
    }
}

// The same in single precision for |x| < 2^23 (a residue times a factor): x (1/p) + 1.5 2^23
// is rounded to 1.5 2^23 + t, whose low 24 bits hold 2^22 + t, and 2^22 p vanishes modulo 2^8.
template <int P>
__device__ __forceinline__ uint32_t crt_small_residue_word(int x) {
    const float tf = __builtin_fmaf((float)x, 1.0f / (float)P, 12582912.0f);
    return __umul24(__float_as_uint(tf), (1u << 24) - (uint32_t)P) + (uint32_t)x;
}

// Recombination of one output matrix: V = sum_i y_i (M / p_i) - t M with t the nearest
// integer to sum_i y_i / p_i, reduced modulo q through w_i = (M / p_i) mod q and M mod q.
struct CrtCombineArgs {
    const uint8_t *Y;    // [D][plane], layout of CrtSeg
    uint64_t *C;
    int64_t m, n, nbc, plane, ldc;
    uint64_t q;
    uint64_t barrett;    // floor(2^64 / q)
    uint64_t Mq;         // M mod q
    uint64_t w[kCrtMaxModuli];  // (M / p_i) mod q; zero past D
    int32_t D, pad;
};

// One operand of a batched residue split: a left operand (rows_side = 1: extent rows of k
// signed values, row stride ld) or a right operand (rows_side = 0: k rows of extent
// residues, row stride ld, centred modulo qc).  Its workgroups are [wg_start, wg_start +
// 128-wide tiles * kblocks).
struct CrtSplitJob {
    int64_t wg_start;
    const void *src;
    int64_t ld, extent, k;
    uint64_t qc;
    int32_t kblocks, rows_side;
    int8_t *out;
};

// A recombination job of a batch: the output matrix's arguments and its first workgroup.
struct CrtCombineJob {
    int64_t wg_start;
    CrtCombineArgs a;
};

// The jobs of one call's splits or recombinations carried in the kernel arguments (no device
// table to allocate or copy): one launch splits up to kCrtTabSplit operands, another
// recombines up to kCrtTabCombine output matrices.
constexpr int kCrtTabSplit = 16;
constexpr int kCrtTabCombine = 8;
// start[j] repeats job[j].wg_start (below 2^31), so that a workgroup finds its job from one
// small scalar load; unused entries hold INT32_MAX.
struct CrtSplitTable {
    int32_t njobs, pad;
    int32_t start[kCrtTabSplit];
    CrtSplitJob job[kCrtTabSplit];
};
struct CrtCombineTable {
    int32_t njobs, pad;
    int32_t start[kCrtTabCombine];
    CrtCombineJob job[kCrtTabCombine];
};

// Factors applied to the left operand's residues in the split: (M / p_i)^{-1} mod p_i.
struct CrtScale {
    int32_t s[kCrtMaxModuli];
};

// One GEMM tile of a multimodular batch, resolved on the host: the first plane blocks of its
// left and right operands for its modulus (k block 0), its k blocks, the modulus, and for
// each of its 128-column plane tiles the product plane that tile writes (blocks per plane
// row, block-column base) or none (null Y).  A tile may straddle the output matrices of one
// problem, which lie side by side in plane tiles, or reach past the last of them.
constexpr int kCrtItemCols = 3;  // plane tiles per batch GEMM tile (384 columns)
struct CrtItem {
    const int8_t *P;
    const int8_t *X;
    uint8_t *Y[kCrtItemCols];
    int64_t nbc[kCrtItemCols];
    int32_t bct[kCrtItemCols];
    int32_t kblocks, p, brt;
};

// Tile classes of the multimodular GEMM (256 x 128, 256 x 256, 256 x 384 outputs); a batch
// runs one persistent GEMM launch per class present.
constexpr int kCrtClasses = 3;

// The items are cut into n_xcd contiguous runs of about equal cost (items differ in K), run x
// being [chunk[x], chunk[x + 1]); XCD x serves run x first, then helps with the others.
struct CrtBatchArgs {
    const CrtItem *items;
    unsigned int *counters;  // one per run, zeroed before each launch: items taken so far
    int64_t total_items;
    int32_t D, n_xcd;
    int64_t chunk[kMaxChunks + 1];
};

}  // namespace hlb
