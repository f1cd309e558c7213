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

// Balanced residue of an integer-valued double |v| < 2^52 modulo p <= 256, in
// [-(p/2), (p-1)/2]: the quotient estimate floor(v / p) is off by at most one, and the fused
// multiply-add forming the remainder is exact.
__device__ __forceinline__ int balanced_residue(double v, int p) {
    const double pd = (double)p;
    const double t = __builtin_floor(v * (1.0 / pd));
    double r = __builtin_fma(-t, pd, v);
    r = r < 0.0 ? r + pd : r;
    r = r >= pd ? r - pd : r;
    const int ri = (int)r;
    return ri >= (p + 1) / 2 ? ri - p : ri;
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

// Factors applied to the left operand's residues in the split: (M / p_i)^{-1} mod p_i.
struct CrtScale {
    int32_t s[kCrtMaxModuli];
};

}  // namespace hlb
