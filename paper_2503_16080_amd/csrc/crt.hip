// crt.hip -- multimodular (CRT) INT8 form of the exact Mod-PP-MM / CP-MM on gfx950.
//
// Strategy 3 of Section 6.1 in its FLINT variant (lift the operands to integers, compute the
// product modulo small coprime moduli, recombine by the CRT), with the moduli chosen so that
// every modular product is one exact INT8 -> INT32 matrix product:
//   1. split: the centred operands (plaintext as signed integers; residues x mod q taken in
//      (-q/2, q/2]) become D planes of balanced residues modulo p_0 .. p_{D-1} <= 256, in the
//      tile-major, swizzled layout of the digit split ([tile][k block][plane][128][64]), the
//      left operand's residues multiplied by (M / p_i)^{-1} mod p_i;
//   2. GEMM: one plain INT8 product per modulus and output tile (v_mfma_i32_32x32x32_i8),
//      |c| <= k 2^14 < 2^31; by the factor above, the byte y_i = c mod p_i is already the
//      CRT coefficient, and the epilogue writes it in the accumulator order (crt.hpp);
//   3. combine: V = sum_i y_i (M / p_i) - t M with t = round(sum_i y_i / p_i) is the exact
//      integer product as long as M > 2 |V|, and V mod q is formed from w_i = (M / p_i) mod q.
// D moduli replace the DP * DX digit products of Strategy 1 (11 instead of 21 for a 20-bit
// plaintext and 50-bit primes at k = 8192; 15 instead of 49 for two full residue operands).
// The splits and recombinations run many operands or output matrices per launch, each
// workgroup finding its job by binary search in a job table (in the kernel arguments for the
// operands of one call, in device memory for a batch); the batch GEMM serves many problems.
#include "common.hpp"
#include "crt.hpp"
#include "crt_jobs.hpp"
#include "launch.hpp"

#include <algorithm>

namespace hlb {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------------------
// 1. Residue split, straight from registers to the workspace (no LDS): one thread owns one
//    16-byte chunk (16 consecutive K) of one row of a 128-row tile -- a row of P, or a
//    column of X -- and writes that chunk of every plane at its swizzled position.  Lanes
//    run over the 4 chunks of a row first, so each 4 lanes store one contiguous 64-byte row.
//    Values are taken as signed integers (qc = 0) or as residues modulo qc in their centred
//    representatives; entries outside the valid range become zero.
// ---------------------------------------------------------------------------------------

// The low bytes of four words as one word (three byte permutes).
__device__ __forceinline__ uint32_t crt_pack4(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3) {
    const uint32_t lo = __builtin_amdgcn_perm(b1, b0, 0x0c0c0400u);  // b0, b1, 0, 0
    const uint32_t hi = __builtin_amdgcn_perm(b3, b2, 0x0c0c0400u);  // b2, b3, 0, 0
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

template <int I, int D, bool SCALED>
__device__ __forceinline__ void crt_store_planes(const CrtValue (&x)[16], int8_t *dst, const CrtScale &scale) {
    if constexpr (I < D) {
        constexpr int p = kCrtModuli[I];
        uint32_t w[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            uint32_t b[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                b[e] = crt_residue_word<p>(x[q4 * 4 + e]);
                // the residue r itself, to scale: for p < 256 the word holds r modulo 2^24 and
                // |r| < 2^7, so its low 24 bits, which the 24-bit multiply reads as a signed
                // number, are r; for p = 256 its byte
                if constexpr (SCALED)
                    b[e] = crt_small_residue_word<p>(p == 256 ? (int)(int8_t)b[e] * scale.s[I] : __mul24((int)b[e], scale.s[I]));
            }
            w[q4] = crt_pack4(b[0], b[1], b[2], b[3]);
        }
        // streaming (non-temporal) stores: the planes are far larger than the caches, and the
        // GEMM that reads them is not slower for it (the split 2-3 % faster)
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(v4u{w[0], w[1], w[2], w[3]}, (v4u *)(dst + I * kCrtR * 64));
        crt_store_planes<I + 1, D, SCALED>(x, dst, scale);
    }
}

// blk: the [D][128][64] block of this (tile, k block); row r, logical chunk c.  With SCALED,
// each residue b becomes the residue of b * s_i (|b s_i| < 2^15).
template <int D, bool SCALED>
__device__ __forceinline__ void crt_store_chunk(const int64_t (&v)[16], int8_t *blk, int r, int c, const CrtScale scale) {
    CrtValue x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = crt_value(v[e]);
    crt_store_planes<0, D, SCALED>(x, blk + r * 64 + ((c ^ swz(r)) << 4), scale);
}

__device__ __forceinline__ int64_t crt_centred(uint64_t x, uint64_t qc) {
    return (qc != 0 && 2 * x > qc) ? (int64_t)x - (int64_t)qc : (int64_t)x;
}

// One (128-row tile, k block) of a left operand: 512 threads = 128 rows x 4 chunks.
template <int D>
__device__ __forceinline__ void crt_split_rows_tile(const int64_t *__restrict__ P, int64_t ldp, int64_t m, int64_t k,
                                                    int kblocks, int tile, int kb, uint64_t qc, const CrtScale &scale,
                                                    int8_t *__restrict__ out) {
    const int r = threadIdx.x >> 2, c = threadIdx.x & 3;
    const int64_t row = (int64_t)tile * kCrtR + r;
    const int64_t k0 = (int64_t)kb * kBK8 + c * 16;
    const int64_t rc = row < m ? row : m - 1;
    uint64_t x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = (uint64_t)P[rc * ldp + (k0 + e < k ? k0 + e : k - 1)];
#pragma unroll
    for (int e = 0; e < 16; ++e) asm volatile("" : "+v"(x[e]));  // all loads issued before the masks
    int64_t v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = (row < m && k0 + e < k) ? crt_centred(x[e], qc) : 0;
    crt_store_chunk<D, true>(v, out + ((int64_t)tile * kblocks + kb) * (D * kCrtR * kBK8), r, c, scale);
}

// One (128-column tile, k block) of a right operand.
template <int D>
__device__ __forceinline__ void crt_split_cols_tile(const uint64_t *__restrict__ X, int64_t ldx, int64_t k, int64_t n,
                                                    int kblocks, int tile, int kb, uint64_t qc,
                                                    int8_t *__restrict__ out) {
    const int r = threadIdx.x >> 2, c = threadIdx.x & 3;
    const int64_t col = (int64_t)tile * kCrtR + r;
    const int64_t k0 = (int64_t)kb * kBK8 + c * 16;
    const int64_t cc = col < n ? col : n - 1;
    uint64_t x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = X[(k0 + e < k ? k0 + e : k - 1) * ldx + cc];
#pragma unroll
    for (int e = 0; e < 16; ++e) asm volatile("" : "+v"(x[e]));
    int64_t v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = (col < n && k0 + e < k) ? crt_centred(x[e], qc) : 0;
    crt_store_chunk<D, false>(v, out + ((int64_t)tile * kblocks + kb) * (D * kCrtR * kBK8), r, c, CrtScale{});
}

// Index of the job owning workgroup w in a table of N start offsets (unused ones INT32_MAX):
// the number of starts <= w, less one.
template <int N>
__device__ __forceinline__ int crt_tab_job(const int32_t (&start)[N], int w) {
    int j = -1;
#pragma unroll
    for (int i = 0; i < N; ++i) j += start[i] <= w;
    return j;
}

// Index of the job owning workgroup w: the last job whose wg_start is <= w (binary search;
// jobs in increasing wg_start, the first at 0).
template <class J>
__device__ __forceinline__ int crt_job_of(const J *__restrict__ jobs, int njobs, int64_t w) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_start <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Many operands in one launch (left operands are scaled by `scale`, right operands centred
// modulo their job's modulus): workgroup w serves the job that owns it.
// Consecutive workgroups take consecutive k blocks of a left operand's row tile (each row's
// bytes are read in order) and consecutive column tiles of a right operand at one k block (each
// row of the operand is read in order across them).
template <int D>
__device__ __forceinline__ void crt_split_job(const CrtSplitJob &j, int64_t w, const CrtScale &scale) {
    const int64_t local = w - j.wg_start;
    if (j.rows_side) {
        const int tile = (int)(local / j.kblocks), kb = (int)(local % j.kblocks);
        crt_split_rows_tile<D>((const int64_t *)j.src, j.ld, j.extent, j.k, j.kblocks, tile, kb, j.qc, scale, j.out);
    } else {
        const int64_t tiles = (j.extent + kCrtR - 1) / kCrtR;
        const int tile = (int)(local % tiles), kb = (int)(local / tiles);
        crt_split_cols_tile<D>((const uint64_t *)j.src, j.ld, j.k, j.extent, j.kblocks, tile, kb, j.qc, j.out);
    }
}

template <int D>
__global__ __launch_bounds__(512) void crt_split_batch(const CrtSplitJob *__restrict__ jobs, int njobs,
                                                       const CrtScale scale) {
    crt_split_job<D>(jobs[crt_job_of(jobs, njobs, blockIdx.x)], blockIdx.x, scale);
}

// The same with the job table in the kernel arguments (the operands of one call).
template <int D>
__global__ __launch_bounds__(512) void crt_split_tab(const CrtSplitTable t, const CrtScale scale) {
    crt_split_job<D>(t.job[crt_tab_job(t.start, (int)blockIdx.x)], blockIdx.x, scale);
}

// ---------------------------------------------------------------------------------------
// 3. Recombination
// ---------------------------------------------------------------------------------------
// x mod q for any x < 2^64 and q < 2^52 (Barrett with mu = floor(2^64 / q): the quotient
// estimate is at most two below floor(x / q), so two corrections finish).
__device__ __forceinline__ uint64_t reduce_u64(uint64_t x, uint64_t q, uint64_t mu) {
    uint64_t r = x - __umul64hi(x, mu) * q;
    r = r >= q ? r - q : r;
    return r >= q ? r - q : r;
}

// Thread: one lane's 16 entries of one 32 x 32 block (16 bytes of every plane, read as one
// 16-byte load each, all issued before any arithmetic); consecutive threads are consecutive
// lanes, so each row of a block is written as 256 contiguous bytes.  For each entry the
// coefficients of four moduli are gathered into one word (a 4 x 4 byte transpose of four
// planes' words), and byte dot products (v_dot4_u32_u8) form
//   L_l = sum_i y_i w_i,l  (w_i,l: byte l of w_i = (M / p_i) mod q, l = 0..6; L_l < 2^20),
//   T   = sum_i y_i c_i    (c_i = round(2^14 / p_i) <= 86).
// S = sum_l L_l 2^(8 l) = sum_i y_i w_i <= 16 * 255 (q - 1), far below 2^64 - q.  The
// rounding t = round(sum_i y_i / p_i) is floor(T / 2^14 + 1/2): the sum lies within 1/4 of
// an integer (the moduli are chosen with M >= 4 |V|), and T / 2^14 differs from it by at most
// sum_i y_i / 2^15 <= 16 * 255 / 2^15 < 1/8.  The output is x mod q for x = S + (-t M mod q),
// with (-t M) mod q from a table in LDS; x < 4081 q, so its quotient has at most 12 bits.
// The estimate floor(x / q - 1/2), formed in single precision (x, 1/q and the product each
// within a few units of 2^-24 relatively: within 0.002 of x / q - 1/2 below 2^12), is
// floor(x / q) or one less, and one conditional subtraction finishes.
__device__ __forceinline__ uint64_t crt_reduce_small_quotient(uint32_t x_lo, uint32_t x_hi, uint64_t q, float qinv) {
    const float xf = __builtin_fmaf((float)x_hi, 4294967296.0f, (float)x_lo);
    const uint32_t qt = (uint32_t)__builtin_fmaxf(__builtin_fmaf(xf, qinv, -0.5f), 0.0f);
    const uint64_t r = (((uint64_t)x_hi << 32) | x_lo) - (uint64_t)qt * q;
    return r >= q ? r - q : r;
}

// The table (-t M) mod q for t = 0 .. D (t <= D since sum_i y_i / p_i < D), in LDS.
__device__ __forceinline__ void crt_negtm_table(const CrtCombineArgs &a, uint64_t *tab) {
    if (threadIdx.x <= (unsigned)a.D) {
        const uint64_t tm = reduce_u64((uint64_t)threadIdx.x * a.Mq, a.q, a.barrett);
        tab[threadIdx.x] = tm == 0 ? 0 : a.q - tm;
    }
    __syncthreads();
}

// c_4g .. c_4g+3 (c_i = round(2^14 / p_i)) as the bytes of one word.
constexpr uint32_t crt_round_word(int g) {
    uint32_t v = 0;
    for (int j = 0; j < 4; ++j) {
        const int p = kCrtModuli[4 * g + j];
        v |= (uint32_t)((32768 + p) / (2 * p)) << (8 * j);
    }
    return v;
}

// Rows a, b, c, d of a 4 x 4 byte matrix (one word each) to its columns: o[j] holds byte j of
// a, b, c and d, in that order.
__device__ __forceinline__ void crt_transpose4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t (&o)[4]) {
    const uint32_t t0 = __builtin_amdgcn_perm(b, a, 0x05010400u);  // a0 b0 a1 b1
    const uint32_t t1 = __builtin_amdgcn_perm(b, a, 0x07030602u);  // a2 b2 a3 b3
    const uint32_t t2 = __builtin_amdgcn_perm(d, c, 0x05010400u);  // c0 d0 c1 d1
    const uint32_t t3 = __builtin_amdgcn_perm(d, c, 0x07030602u);  // c2 d2 c3 d3
    o[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    o[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    o[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    o[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// The 16 entries of one lane of block (br, bc), for G groups of four moduli (4 G >= D; the
// planes past D read as zero).  CHECK: some rows of the block lie past m.
template <int G, bool CHECK>
__device__ __forceinline__ void crt_combine_entries(const CrtCombineArgs &a, const uint64_t *tab, int64_t br,
                                                    int64_t bc, int lane) {
    const uint8_t *y = a.Y + ((br * a.nbc + bc) * 64 + lane) * 16;
    uint4 v[4 * G];
#pragma unroll
    for (int i = 0; i < 4 * G; ++i) {
        if (i < 4 * (G - 1) || i < a.D) v[i] = *(const uint4 *)(y + (int64_t)i * a.plane);
        else v[i] = uint4{0u, 0u, 0u, 0u};
    }
    // byte l of w_4g .. w_4g+3 as one word (uniform; w_i = 0 past D)
    uint32_t wl[7][G];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int l = 0; l < 7; ++l) {
            uint32_t word = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) word |= (uint32_t)((a.w[4 * g + j] >> (8 * l)) & 0xffu) << (8 * j);
            wl[l][g] = word;
        }
    const float qinv = 1.0f / (float)a.q;
    const int64_t row0 = br * 32 + 4 * (lane >> 5);
    uint64_t *out = a.C + row0 * a.ldc + bc * 32 + (lane & 31);  // advanced row by row below
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // word k of each plane: entries 4 k .. 4 k + 3
        uint32_t yt[4][G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t wa[4] = {v[4 * g].x, v[4 * g].y, v[4 * g].z, v[4 * g].w};
            const uint32_t wb[4] = {v[4 * g + 1].x, v[4 * g + 1].y, v[4 * g + 1].z, v[4 * g + 1].w};
            const uint32_t wc[4] = {v[4 * g + 2].x, v[4 * g + 2].y, v[4 * g + 2].z, v[4 * g + 2].w};
            const uint32_t wd[4] = {v[4 * g + 3].x, v[4 * g + 3].y, v[4 * g + 3].z, v[4 * g + 3].w};
            uint32_t o[4];
            crt_transpose4(wa[k], wb[k], wc[k], wd[k], o);
#pragma unroll
            for (int b = 0; b < 4; ++b) yt[b][g] = o[b];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {  // entry 4 k + b: row 8 k + b of this lane's half-block
            uint32_t L[7], T = 0;
#pragma unroll
            for (int l = 0; l < 7; ++l) L[l] = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
#pragma unroll
                for (int l = 0; l < 7; ++l) L[l] = __builtin_amdgcn_udot4(yt[b][g], wl[l][g], L[l], false);
                T = __builtin_amdgcn_udot4(yt[b][g], crt_round_word(g), T, false);
            }
            // x = S + (-t M mod q) as two words: S = lo + mid 2^16 + hi 2^32 with lo, mid < 2^29
            // and hi < 2^32 (S < 2^64); no carry leaves the high word (x < 2^64)
            const uint32_t lo = L[0] + (L[1] << 8), mid = L[2] + (L[3] << 8), hi = L[4] + (L[5] << 8) + (L[6] << 16);
            const uint64_t e = tab[(T + 8192u) >> 14];
            uint32_t c0, c1;
            const uint32_t s_lo = __builtin_addc(lo, mid << 16, 0u, &c0);
            const uint32_t x_lo = __builtin_addc(s_lo, (uint32_t)e, 0u, &c1);
            const uint32_t x_hi = (mid >> 16) + hi + (uint32_t)(e >> 32) + c0 + c1;
            const uint64_t r = crt_reduce_small_quotient(x_lo, x_hi, a.q, qinv);
            if (!CHECK || row0 + 8 * k + b < a.m) __builtin_nontemporal_store(r, out);  // streaming store
            out += b < 3 ? a.ldc : 5 * a.ldc;
        }
    }
}

// Many output matrices in one launch: each workgroup serves kThreads / 64 blocks of the job
// that owns it, one per wave (the block index is uniform over a wave).
__device__ __forceinline__ void crt_combine_job(const CrtCombineJob &j, uint64_t *tab) {
    const CrtCombineArgs &a = j.a;
    crt_negtm_table(a, tab);
    const int64_t nbc_valid = (a.n + 31) >> 5;
    const int64_t blocks = ((a.m + 31) >> 5) * nbc_valid;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t blk = ((int64_t)blockIdx.x - j.wg_start) * (kThreads / 64) + wave;
    if (blk >= blocks) return;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t br = blk / nbc_valid, bc = blk - br * nbc_valid;
    if (bc * 32 + (lane & 31) >= a.n) return;
    const bool full = br * 32 + 32 <= a.m;
    if (a.D <= 8) {
        if (full) crt_combine_entries<2, false>(a, tab, br, bc, lane);
        else crt_combine_entries<2, true>(a, tab, br, bc, lane);
    } else if (a.D <= 12) {
        if (full) crt_combine_entries<3, false>(a, tab, br, bc, lane);
        else crt_combine_entries<3, true>(a, tab, br, bc, lane);
    } else {
        if (full) crt_combine_entries<4, false>(a, tab, br, bc, lane);
        else crt_combine_entries<4, true>(a, tab, br, bc, lane);
    }
}

__global__ __launch_bounds__(kThreads) void crt_combine_batch(const CrtCombineJob *__restrict__ jobs, int njobs) {
    __shared__ uint64_t tab[kCrtMaxModuli + 1];
    crt_combine_job(jobs[crt_job_of(jobs, njobs, blockIdx.x)], tab);
}

// The same with the job table in the kernel arguments (the outputs of one call).
__global__ __launch_bounds__(kThreads) void crt_combine_tab(const CrtCombineTable t) {
    __shared__ uint64_t tab[kCrtMaxModuli + 1];
    crt_combine_job(t.job[crt_tab_job(t.start, (int)blockIdx.x)], tab);
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
bool crt_supported_d(int D) { return D == 8 || D == 10 || D == 11 || D == 12 || D == 14 || D == 16; }

int crt_round_d(int D) {
    for (int d : {8, 10, 11, 12, 14, 16})
        if (D <= d) return d;
    return 0;
}

#define HLB_CRT_D(X) X(8) X(10) X(11) X(12) X(14) X(16)

int64_t crt_combine_wgs(int64_t m, int64_t n) { return (((m + 31) / 32) * ((n + 31) / 32) * 64 + kThreads - 1) / kThreads; }

hipError_t launch_crt_split_batch(int D, const CrtSplitJob *jobs, int njobs, int64_t total_wgs, const CrtScale &scale,
                                  hipStream_t s) {
    if (total_wgs <= 0 || njobs <= 0) return hipSuccess;
    if (total_wgs > INT32_MAX) return hipErrorInvalidValue;
    const dim3 g((unsigned)total_wgs), b(512);
#define HLB_CASE(DD) \
    if (D == DD) { hipLaunchKernelGGL(crt_split_batch<DD>, g, b, 0, s, jobs, njobs, scale); return hipGetLastError(); }
    HLB_CRT_D(HLB_CASE)
#undef HLB_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_crt_split_tab(int D, const CrtSplitTable &t, int64_t total_wgs, const CrtScale &scale,
                                hipStream_t s) {
    if (total_wgs <= 0 || t.njobs <= 0) return hipSuccess;
    if (total_wgs > INT32_MAX || t.njobs > kCrtTabSplit) return hipErrorInvalidValue;
    const dim3 g((unsigned)total_wgs), b(512);
#define HLB_CASE(DD) \
    if (D == DD) { hipLaunchKernelGGL(crt_split_tab<DD>, g, b, 0, s, t, scale); return hipGetLastError(); }
    HLB_CRT_D(HLB_CASE)
#undef HLB_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_crt_combine_tab(const CrtCombineTable &t, int64_t total_wgs, hipStream_t s) {
    if (total_wgs <= 0 || t.njobs <= 0) return hipSuccess;
    if (total_wgs > INT32_MAX || t.njobs > kCrtTabCombine) return hipErrorInvalidValue;
    hipLaunchKernelGGL(crt_combine_tab, dim3((unsigned)total_wgs), dim3(kThreads), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_crt_combine_batch(const CrtCombineJob *jobs, int njobs, int64_t total_wgs, hipStream_t s) {
    if (total_wgs <= 0 || njobs <= 0) return hipSuccess;
    if (total_wgs > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(crt_combine_batch, dim3((unsigned)total_wgs), dim3(kThreads), 0, s, jobs, njobs);
    return hipGetLastError();
}

}  // namespace hlb
