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
template <int D>
__device__ __forceinline__ void crt_split_job(const CrtSplitJob &j, int64_t w, const CrtScale &scale) {
    const int64_t local = w - j.wg_start;
    const int tile = (int)(local / j.kblocks), kb = (int)(local % j.kblocks);
    if (j.rows_side)
        crt_split_rows_tile<D>((const int64_t *)j.src, j.ld, j.extent, j.k, j.kblocks, tile, kb, j.qc, scale, j.out);
    else
        crt_split_cols_tile<D>((const uint64_t *)j.src, j.ld, j.k, j.extent, j.kblocks, tile, kb, j.qc, j.out);
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
// 16-byte load each); consecutive threads are consecutive lanes, so each row of a block is
// written as 256 contiguous bytes.  S = sum_i y_i w_i < 16 * 2^8 * 2^52 is accumulated in
// three 20-bit limbs of w_i (each limb sum stays below 2^32, 24-bit multiply-adds), and the
// rounding t = round(sum_i y_i / p_i) needs only single precision: the fraction lies within
// 1/4 of an integer, far beyond its rounding error.  (t M) mod q comes from a table in LDS.
__device__ __forceinline__ void crt_tmq_table(const CrtCombineArgs &a, uint64_t *tmq) {
    if (threadIdx.x <= (unsigned)a.D) tmq[threadIdx.x] = reduce_u64((uint64_t)threadIdx.x * a.Mq, a.q, a.barrett);
    __syncthreads();
}

// Entries g of one output matrix (g = 64 * (32 x 32 block) + lane, g < 64 * blocks).
__device__ __forceinline__ void crt_combine_lane(const CrtCombineArgs &a, const uint64_t *tmq, int64_t g,
                                                 int64_t nbc_valid) {
    const int lane = (int)(g & 63);
    const int64_t b = g >> 6, br = b / nbc_valid, bc = b - br * nbc_valid;
    const uint8_t *y = a.Y + ((br * a.nbc + bc) * 64 + lane) * 16;
    uint32_t s0[16], s1[16], s2[16];
    float f[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        s0[e] = s1[e] = s2[e] = 0u;
        f[e] = 0.f;
    }
#pragma unroll 2
    for (int i = 0; i < a.D; ++i) {
        const uint4 v = *(const uint4 *)(y + (int64_t)i * a.plane);
        const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
        const uint64_t w = a.w[i];
        const uint32_t w0 = (uint32_t)w & 0xfffffu, w1 = (uint32_t)(w >> 20) & 0xfffffu, w2 = (uint32_t)(w >> 40);
        const float pi = a.pinv[i];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t byte = (vw[e >> 2] >> (8 * (e & 3))) & 0xffu;
            s0[e] += __umul24(byte, w0);
            s1[e] += __umul24(byte, w1);
            s2[e] += __umul24(byte, w2);
            f[e] = __builtin_fmaf((float)byte, pi, f[e]);
        }
    }
    const int64_t col = bc * 32 + (lane & 31);
    if (col >= a.n) return;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t row = br * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (row >= a.m) continue;
        const uint64_t sum = ((uint64_t)s2[e] << 40) + ((uint64_t)s1[e] << 20) + s0[e];
        const uint64_t sr = reduce_u64(sum, a.q, a.barrett);
        const uint64_t tm = tmq[(int)__builtin_floorf(f[e] + 0.5f)];
        // streaming store: the outputs are not read again here
        __builtin_nontemporal_store(sr >= tm ? sr - tm : sr + a.q - tm, &a.C[row * a.ldc + col]);
    }
}

// Many output matrices in one launch: each workgroup serves kThreads entry groups of the job
// that owns it.
__device__ __forceinline__ void crt_combine_job(const CrtCombineJob &j, uint64_t *tmq) {
    crt_tmq_table(j.a, tmq);
    const int64_t nbc_valid = (j.a.n + 31) >> 5;
    const int64_t total = ((j.a.m + 31) >> 5) * nbc_valid * 64;
    const int64_t g = ((int64_t)blockIdx.x - j.wg_start) * kThreads + threadIdx.x;
    if (g < total) crt_combine_lane(j.a, tmq, g, nbc_valid);
}

__global__ __launch_bounds__(kThreads) void crt_combine_batch(const CrtCombineJob *__restrict__ jobs, int njobs) {
    __shared__ uint64_t tmq[kCrtMaxModuli + 1];
    crt_combine_job(jobs[crt_job_of(jobs, njobs, blockIdx.x)], tmq);
}

// The same with the job table in the kernel arguments (the outputs of one call).
__global__ __launch_bounds__(kThreads) void crt_combine_tab(const CrtCombineTable t) {
    __shared__ uint64_t tmq[kCrtMaxModuli + 1];
    crt_combine_job(t.job[crt_tab_job(t.start, (int)blockIdx.x)], tmq);
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
