// crt.hpp -- moduli and argument structures of the multimodular (CRT) INT8 form.
//
// Strategy 3 of Section 6.1 in the variant the paper attributes to FLINT: instead of
// modulus-switching the ciphertext, the product P X of the centred integer operands is
// computed modulo pairwise coprime small moduli p_0 .. p_{D-1} whose product M exceeds twice
// its magnitude, and is recovered by the CRT.  Moduli up to 256 keep the balanced residues
// in [-128, 127], so each product modulo p_i is one exact INT8 -> INT32 matrix product.
#pragma once

#include <stdint.h>

#include "common.hpp"

namespace hlb {

constexpr int kCrtMaxModuli = 16;
// Pairwise coprime, descending: 2^8, 3*5*17, 11*23, 251, 13*19, then primes.
constexpr int kCrtModuli[kCrtMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233,
                                           229, 227, 223, 211, 199, 197, 193, 191};

constexpr int crt_pow2_mod(int e, int p) {
    int r = 1 % p;
    for (int i = 0; i < e; ++i) r = (2 * r) % p;
    return r;
}

// A signed integer |s| < 2^52 as s = a 2^32 + b 2^16 + c with |a| <= 2^20, 0 <= b, c < 2^16.
struct CrtPieces {
    int a, b, c;
};
__device__ __forceinline__ CrtPieces crt_pieces(int64_t s) {
    return {(int)(s >> 32), (int)(((uint64_t)s >> 16) & 0xffffu), (int)((uint64_t)s & 0xffffu)};
}

// Balanced residue of an integer |u| < 2^29 modulo p <= 256, in [-(p/2), (p-1)/2]: the
// nearest-integer quotient estimate from single precision is off by at most one (|u| / p
// carries an error below 0.3), and one correction each way removes that.
__device__ __forceinline__ int crt_balanced(int u, int p, float pinv) {
    const int t = (int)__builtin_floorf(__builtin_fmaf((float)u, pinv, 0.5f));
    int r = u - __mul24(t, p);
    r = r > (p - 1) / 2 ? r - p : r;
    return r < -(p / 2) ? r + p : r;
}

// Balanced residue of the pieces modulo the i-th modulus: a (2^32 mod p) + b (2^16 mod p) + c
// is congruent to s and below 2^28.1 in magnitude.
template <int I>
__device__ __forceinline__ int crt_residue(const CrtPieces &x) {
    constexpr int p = kCrtModuli[I];
    constexpr int e32 = crt_pow2_mod(32, p), e16 = crt_pow2_mod(16, p);
    return crt_balanced(__mul24(x.a, e32) + __mul24(x.b, e16) + x.c, p, 1.0f / (float)p);
}

// Product planes.  The GEMM of modulus i writes y_i = C_i mod p_i as one byte per entry (the
// left operand's residues carry the factor (M / p_i)^{-1}, so y_i is already the CRT
// coefficient).  A plane covers the output padded to whole GEMM tiles and is stored in the
// accumulator order of v_mfma_i32_32x32x32_i8: 32 x 32 blocks, row-major over the padded grid,
// each block as 64 lanes x 16 bytes, where lane l, byte r holds row 8 (r / 4) + 4 (l / 32) +
// r % 4 and column l % 32 of the block.  Each lane thus stores its 16 results as one
// contiguous 16-byte write.
struct CrtSeg {
    uint8_t *Y;          // [D][plane] bytes of this output matrix
    int64_t n;           // valid columns
    int64_t nbc;         // 32-column blocks per padded row
    int64_t plane;       // bytes per modulus: padded rows x padded columns
    int32_t tile_begin;  // first global GEMM column tile
    int32_t pad;
};

struct CrtGemmArgs {
    const int8_t *Pd;    // left operand planes: [128-row tile][k block][D][128][64]
    const int8_t *Xd;    // right operand planes: [128-col tile][k block][D][128][64]
    int64_t m;
    int32_t kblocks, D;
    int32_t tiles_m;     // 256-row tiles
    int32_t tiles_n;     // GEMM column tiles (128 or 256 wide) over all segments
    int32_t group_m, n_xcd, nseg, pad;
    CrtSeg seg[kMaxSegs];
};

// Recombination of one output matrix: V = sum_i y_i (M / p_i) - t M with t the nearest
// integer to sum_i y_i / p_i, reduced modulo q through w_i = (M / p_i) mod q and M mod q.
struct CrtCombineArgs {
    const uint8_t *Y;    // [D][plane], layout of CrtSeg
    uint64_t *C;
    int64_t m, n, nbc, plane, ldc;
    uint64_t q;
    uint64_t barrett;    // floor(2^64 / q)
    uint64_t Mq;         // M mod q
    uint64_t w[kCrtMaxModuli];
    float pinv[kCrtMaxModuli];  // 1 / p_i
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

// One GEMM tile of a multimodular batch, resolved on the host: the first plane blocks of its
// left and right operands for its modulus (k block 0), its k blocks, the modulus, and the
// product plane it writes (block-row and block-column bases, blocks per plane row).
struct CrtItem {
    const int8_t *P;
    const int8_t *X;
    uint8_t *Y;
    int64_t nbc;
    int32_t kblocks, p, brt, bct;
};

// The items are cut into n_xcd contiguous runs of about equal cost (items differ in K), run x
// being [chunk[x], chunk[x + 1]); XCD x serves run x.
struct CrtBatchArgs {
    const CrtItem *items;
    int64_t total_items;
    int32_t D, n_xcd;
    int64_t chunk[kMaxChunks + 1];
};

// A recombination job of a batch: the output matrix's arguments and its first workgroup.
struct CrtCombineJob {
    int64_t wg_start;
    CrtCombineArgs a;
};

// Factors applied to the left operand's residues in the split: (M / p_i)^{-1} mod p_i.
struct CrtScale {
    int32_t s[kCrtMaxModuli];
};

}  // namespace hlb
