// split.hpp -- the split of an operand into int8 planes in the tile-major workspace layout.
//
// One workgroup handles one (tile, k block): R rows (plaintext side) or R columns
// (ciphertext side, transposed) by 64 K elements.  A converter turns 4 consecutive K
// elements of a row into D packed dwords, one per plane (byte e of dword j = plane j of
// element e): balanced base-256 digits for Strategy 1, balanced residues modulo small
// moduli for the multimodular form.
#pragma once

#include "common.hpp"

namespace hlb {

// ---------------------------------------------------------------------------------------
// Digit split.  One workgroup per (tile row, k block): R rows x 64 K elements.
//   Stage 1: each thread loads 4 consecutive K elements of one row (plaintext side: a row
//            of P; ciphertext side: a column of X, read as 4 rows of X at one column so
//            that lanes with consecutive columns load consecutive addresses), splits them
//            into D digits and writes one dword (4 digit bytes) per digit into LDS.
//   Stage 2: 16-byte chunks are copied from LDS to the swizzled tile-major workspace.
// Entries outside the valid m x k (or k x n) range become zero digits.
// ---------------------------------------------------------------------------------------
constexpr int kSplitRowPad = 68;  // LDS row stride in bytes: 64 + 4 keeps dword writes conflict-free
constexpr int kSplitLds = 7 * 128 * kSplitRowPad;  // LDS of the largest digit split

// Keeps the compiler from turning a load whose value a later select may discard back into
// a conditional load (a branch per element, each waiting for its load): the empty asm
// consumes every loaded value unconditionally, after all the loads have been issued.
template <int N>
__device__ __forceinline__ void pin_loaded(uint64_t (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]));
}

// Balanced base-256 digits: plane j of 4 values packed into one dword (byte e = value e).
template <int D>
struct DigitConv {
    __device__ __forceinline__ void operator()(const uint64_t (&x)[4], uint32_t (&out)[D]) const {
        constexpr uint64_t bias = digit_bias(D);
        uint64_t y[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) y[e] = x[e] + bias;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            uint32_t w = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) w |= (uint32_t)((y[e] >> (8 * j)) & 0xffu) << (8 * e);
            out[j] = w ^ 0x80808080u;
        }
    }
};

template <int D, int R>
__device__ __forceinline__ void split_stage2(const uint8_t *lds, int8_t *tile_out) {
    constexpr int chunks = D * R * 4;
    static_assert(chunks % kThreads == 0, "tile chunks must divide evenly");
#pragma unroll
    for (int it = 0; it < chunks / kThreads; ++it) {
        const int ci = threadIdx.x + it * kThreads;
        const int j = ci / (R * 4);
        const int r = (ci / 4) % R;
        const int c = ci % 4;
        const uint32_t *src = (const uint32_t *)(lds + (j * R + r) * kSplitRowPad + c * 16);
        uint4 v;
        v.x = src[0];
        v.y = src[1];
        v.z = src[2];
        v.w = src[3];
        // logical chunk c of row r lives at physical chunk c ^ swz(r)
        *(uint4 *)(tile_out + (j * R + r) * 64 + ((c ^ swz(r)) << 4)) = v;
    }
}

// One (row tile rb, k block kb) of the plaintext side: rows of P (signed int64 or residues).
// Every thread first issues all its loads (4 consecutive K elements of R/16 rows), from
// clamped in-bounds addresses, and only then masks and splits them: a conditional load
// would become a branch that waits for each load before issuing the next.
template <int D, int R, class Conv>
__device__ __forceinline__ void split_rows_tile(const int64_t *__restrict__ P, int64_t ldp, int64_t m,
                                                int64_t k, int kblocks, int rb, int kb, int8_t *out,
                                                uint8_t *lds, const Conv &conv) {
    constexpr int IT = R / (kThreads / 16);
    const int t = threadIdx.x;
    const int quad = t & 15;  // 4 consecutive K elements
    const int64_t k0 = (int64_t)kb * kBK8 + quad * 4;
    uint64_t x[IT][4];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int64_t row = (int64_t)rb * R + (t >> 4) + it * (kThreads / 16);
        const int64_t rc = row < m ? row : m - 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[it][e] = (uint64_t)P[rc * ldp + (k0 + e < k ? k0 + e : k - 1)];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) pin_loaded(x[it]);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int r = (t >> 4) + it * (kThreads / 16);
        const int64_t row = (int64_t)rb * R + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[it][e] = (row < m && k0 + e < k) ? x[it][e] : 0;
        uint32_t d[D];
        conv(x[it], d);
#pragma unroll
        for (int j = 0; j < D; ++j) *(uint32_t *)(lds + (j * R + r) * kSplitRowPad + quad * 4) = d[j];
    }
    __syncthreads();
    split_stage2<D, R>(lds, out + ((int64_t)rb * kblocks + kb) * (D * R * kBK8));
}

// One (column tile cb, k block kb) of the ciphertext side: columns of X (transposed).  Each
// lane owns one column and loads 4 consecutive rows at a time, so lanes with consecutive
// columns read consecutive addresses; loads are issued first as above.
template <int D, int R, class Conv>
__device__ __forceinline__ void split_cols_tile(const uint64_t *__restrict__ X, int64_t ldx, int64_t k,
                                                int64_t n, int kblocks, int cb, int kb, int8_t *out,
                                                uint8_t *lds, const Conv &conv) {
    constexpr int quads_in_flight = kThreads / R;  // K quads handled per pass
    constexpr int IT = 16 / quads_in_flight;
    const int t = threadIdx.x;
    const int c = t % R;
    const int64_t col = (int64_t)cb * R + c;
    const int64_t cc = col < n ? col : n - 1;
    uint64_t x[IT][4];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int64_t k0 = (int64_t)kb * kBK8 + (t / R + it * quads_in_flight) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[it][e] = X[(k0 + e < k ? k0 + e : k - 1) * ldx + cc];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) pin_loaded(x[it]);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int qd = t / R + it * quads_in_flight;
        const int64_t k0 = (int64_t)kb * kBK8 + qd * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[it][e] = (col < n && k0 + e < k) ? x[it][e] : 0;
        uint32_t d[D];
        conv(x[it], d);
#pragma unroll
        for (int j = 0; j < D; ++j) *(uint32_t *)(lds + (j * R + c) * kSplitRowPad + qd * 4) = d[j];
    }
    __syncthreads();
    split_stage2<D, R>(lds, out + ((int64_t)cb * kblocks + kb) * (D * R * kBK8));
}

}  // namespace hlb
