// crt.hpp -- moduli, plane layout and GEMM arguments of the multimodular (CRT) INT8 form.
//
// Strategy 3 of Section 6.1 in the variant the paper attributes to FLINT: instead of
// modulus-switching the ciphertext, the product P X of the centred integer operands is
// computed modulo pairwise coprime small moduli p_0 .. p_{D-1} whose product M exceeds twice
// its magnitude, and is recovered by the CRT.  Moduli up to 256 keep the balanced residues
// in [-128, 127], so each product modulo p_i is one exact INT8 -> INT32 matrix product
// (crt_gemm.hip).  The splits and the recombination are declared in crt_jobs.hpp.
#pragma once

#include <stdint.h>

#include "common.hpp"

namespace hlb {

constexpr int kCrtMaxModuli = 16;
// Pairwise coprime, descending: 2^8, 3*5*17, 11*23, 251, 13*19, then primes.
constexpr int kCrtModuli[kCrtMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233,
                                           229, 227, 223, 211, 199, 197, 193, 191};

// Residue planes are stored in tiles of 128 rows of the left operand (or 128 columns of the
// right operand, transposed) by 64 K bytes: [tile][k block][modulus][128][64].
constexpr int kCrtR = 128;

// Product planes.  The GEMM of modulus i writes y_i = C_i mod p_i as one byte per entry (the
// left operand's residues carry the factor (M / p_i)^{-1}, so y_i is already the CRT
// coefficient).  A plane covers the output with its rows padded to whole 256-row GEMM tiles
// and its columns to whole 128-column plane tiles, and is stored in the accumulator order of
// v_mfma_i32_32x32x32_i8: 32 x 32 blocks, row-major over the padded grid, each block as 64
// lanes x 16 bytes, where lane l, byte r holds row 8 (r / 4) + 4 (l / 32) + r % 4 and column
// l % 32 of the block.  Each lane thus stores its 16 results as one contiguous 16-byte write.
struct CrtSeg {
    uint8_t *Y;          // [D][plane] bytes of this output matrix
    int64_t n;           // valid columns
    int64_t nbc;         // 32-column blocks per padded row
    int64_t plane;       // bytes per modulus: padded rows x padded columns
    int32_t tile_begin;  // first 128-column plane tile of this matrix among the launch's
    int32_t tiles;       // and their count: the launch's matrices lie side by side
};

struct CrtGemmArgs {
    const int8_t *Pd;    // left operand planes: [128-row tile][k block][D][128][64]
    const int8_t *Xd;    // right operand planes: [128-col tile][k block][D][128][64]
    int64_t m;
    int32_t kblocks, D;
    int32_t tiles_m;     // 256-row tiles
    int32_t tiles_n;     // GEMM column tiles (128, 256 or 384 wide) over all segments, which
                         // may straddle two segments
    int32_t group_m, n_xcd, nseg, pad;
    unsigned int *counters;  // kMaxChunks tile-queue counters of a persistent launch, or null
    CrtSeg seg[kMaxSegs];
};

}  // namespace hlb
