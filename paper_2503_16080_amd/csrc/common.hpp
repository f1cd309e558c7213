// common.hpp -- shared definitions of the libhlb device code (gfx950 only).
//
// Tile geometry, the digit-plane workspace layout, modular arithmetic helpers and the kernel
// argument structures used by the split kernels, the limb GEMMs and the host dispatcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlb {

// ---------------------------------------------------------------------------------------
// Limits
// ---------------------------------------------------------------------------------------
constexpr int kMaxSegs = 16;          // output matrices (prime x part) per GEMM launch
constexpr int kThreads = 256;         // 4 waves of 64 per workgroup, arranged 2 x 2
constexpr int kBK8 = 64;              // K bytes per LDS stage (INT8 form)
constexpr int kBK64 = 16;             // K elements per LDS stage (FP64 form)
constexpr uint64_t kMaxModulus = (uint64_t)1 << 52;

// ---------------------------------------------------------------------------------------
// Digit-plane workspace layout (INT8 form).
//
// A matrix split into D balanced int8 digits is stored tile-major so that one LDS stage of
// one workgroup is a single contiguous block:  [tile_row][k_block][digit][R][64 bytes],
// where R (= BM for the plaintext side, BN for the ciphertext side) rows of 64 consecutive
// K bytes form one digit plane of the tile.  For the ciphertext side a "row" is a column
// of X (the split transposes), so both MFMA operands are K-contiguous.  Inside a row the
// four 16-byte chunks are XOR-swizzled by swz(row) so that the MFMA fragment reads
// (32 rows x one 16-byte chunk per wave) hit distinct LDS banks.
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// Balanced digits: x = sum_j d_j 256^j with d_j in [-128, 127].  Adding the bias
// C_D = sum_{j<D} 128 * 256^j turns them into plain bytes u_j = d_j + 128 of x + C_D, so the
// digits are the bytes of (x + C_D) with the top bit flipped.  x is representable with D
// digits iff 0 <= x + C_D < 256^D.
__host__ __device__ constexpr uint64_t digit_bias(int D) {
    uint64_t c = 0;
    for (int j = 0; j < D; ++j) c |= (uint64_t)0x80 << (8 * j);
    return c;
}

// ---------------------------------------------------------------------------------------
// Modular arithmetic (device).  q < 2^52 throughout.
// ---------------------------------------------------------------------------------------

// Canonical t mod q for a signed t with |t| < 2^62 and |t / q| < 2^49.  The quotient
// estimate floor(t * (1/q)) carries three double roundings (relative error <= 3 * 2^-53),
// so it is off by at most one and a single correction in each direction lands in [0, q).
// Branch-free (selects only), so callers can be fully unrolled over register arrays.
__device__ __forceinline__ uint64_t reduce_near(int64_t t, uint64_t q, double qinv) {
    const double est = __builtin_floor((double)t * qinv);
    int64_t r = t - (int64_t)est * (int64_t)q;
    r = r < 0 ? r + (int64_t)q : r;
    r = r >= (int64_t)q ? r - (int64_t)q : r;
    return (uint64_t)r;
}

// Canonical c mod q for an integer-valued double c.  The estimate est = floor(c * (1/q))
// carries two roundings (relative error <= 2^-52), so est is within |c/q| 2^-52 + 1 of c/q:
//  * |c| < 2^53: est is off by at most two and the exact remainder c - est * q lies in
//    (-2q, 3q); for q >= 2^51 the error is < 2^-50 and it lies in [-q, 2q);
//  * |c| < q 2^51 (any magnitude of c/q up to 2^51): est is off by at most one and the
//    remainder lies in [-q, 2q).
// Either way it is an integer below 2^53 in magnitude, so the fused multiply-add that forms
// it rounds nothing, and two corrections each way finish.
__device__ __forceinline__ uint64_t reduce_fp(double c, uint64_t q, double qd, double qinv) {
    const double est = __builtin_floor(c * qinv);
    double r = __builtin_fma(-est, qd, c);
    r = r < 0.0 ? r + qd : r;
    r = r < 0.0 ? r + qd : r;
    r = r >= qd ? r - qd : r;
    r = r >= qd ? r - qd : r;
    return (uint64_t)r;
}

// a * w mod q for a constant w < q with Shoup companion wp = floor(w * 2^64 / q);
// valid for any a < 2^64 (the result of the two wrapping products lies in [0, 2q)).
__device__ __forceinline__ uint64_t mulmod_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    const uint64_t hi = __umul64hi(a, wp);
    const uint64_t r = a * w - hi * q;
    return r >= q ? r - q : r;
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    const uint64_t s = a + b;
    return s >= q ? s - q : s;
}

// ---------------------------------------------------------------------------------------
// LDS pipelines fed by direct-to-LDS global loads
// ---------------------------------------------------------------------------------------

// A buffer resource over a wave-uniform base, for the copies below.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t lds_src_rsrc(const int8_t *base) {
    // the base is wave-uniform; say so, so that the descriptor lives in scalar registers
    const uint64_t p = (uint64_t)(uintptr_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(uintptr_t)(((uint64_t)hi << 32) | lo), 0, 0xffffffff,
                                             0x00020000);
}
// Copies CHUNKS 16-byte chunks from global memory to LDS with the buffer form of the gfx950
// direct-to-LDS load (MUBUF ... lds): lane l of a wave writes its 16 bytes at (wave-uniform LDS
// base) + 16 l, so the linear chunk order of the tile-major workspace arrives unchanged and no
// staging registers are used; chunks are dealt to waves in runs of 64.  The source is `rsrc`
// + src_off, byte offsets below 2^32.  The compiler counts these loads in vmcnt only (the
// global form also counts as an LDS event, which makes every LDS read wait for all of them),
// so LDS fragment reads after them can wait for just the reads they need.  src_off is
// wave-uniform and goes in the scalar offset; the per-lane offset is the same for every stage
// and block, so one register serves all loads.
template <int THREADS, int CHUNKS>
__device__ __forceinline__ void copy_to_lds_buf(__amdgpu_buffer_rsrc_t rsrc, uint32_t src_off, int8_t *dst, int tid,
                                                int wave_u) {
#pragma unroll
    for (int i = 0; i < (CHUNKS + THREADS - 1) / THREADS; ++i) {
        const int base = i * THREADS + wave_u * 64;  // wave-uniform
        if (CHUNKS % THREADS == 0 || base < CHUNKS)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void *)(dst + base * 16),
                                                     16, (uint32_t)(i * THREADS + tid) * 16u,
                                                     __builtin_amdgcn_readfirstlane(src_off), 0, 0);
    }
}

// Direct-to-LDS loads a wave issues for one stage (chunks are dealt in runs of 64).
template <int THREADS, int CHUNKS>
__device__ __forceinline__ int loads_of_wave(int wave_u) {
    int n = 0;
#pragma unroll
    for (int i = 0; i < (CHUNKS + THREADS - 1) / THREADS; ++i) n += (i * THREADS + wave_u * 64 < CHUNKS);
    return n;
}

// s_waitcnt vmcnt(n) for a wave-uniform n known only at run time (the immediate must be a
// constant, so the possible counts are enumerated).
__device__ __forceinline__ void wait_vmcnt(int n) {
    switch (n) {
        case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
        case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
        case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
        case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
        case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
        case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
        case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
        case 7: asm volatile("s_waitcnt vmcnt(7)" ::: "memory"); break;
        case 8: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
        case 9: asm volatile("s_waitcnt vmcnt(9)" ::: "memory"); break;
        case 10: asm volatile("s_waitcnt vmcnt(10)" ::: "memory"); break;
        case 11: asm volatile("s_waitcnt vmcnt(11)" ::: "memory"); break;
        case 12: asm volatile("s_waitcnt vmcnt(12)" ::: "memory"); break;
        case 13: asm volatile("s_waitcnt vmcnt(13)" ::: "memory"); break;
        case 14: asm volatile("s_waitcnt vmcnt(14)" ::: "memory"); break;
        case 15: asm volatile("s_waitcnt vmcnt(15)" ::: "memory"); break;
        case 16: asm volatile("s_waitcnt vmcnt(16)" ::: "memory"); break;
        case 17: asm volatile("s_waitcnt vmcnt(17)" ::: "memory"); break;
        case 18: asm volatile("s_waitcnt vmcnt(18)" ::: "memory"); break;
        case 19: asm volatile("s_waitcnt vmcnt(19)" ::: "memory"); break;
        case 20: asm volatile("s_waitcnt vmcnt(20)" ::: "memory"); break;
        case 21: asm volatile("s_waitcnt vmcnt(21)" ::: "memory"); break;
        case 22: asm volatile("s_waitcnt vmcnt(22)" ::: "memory"); break;
        case 23: asm volatile("s_waitcnt vmcnt(23)" ::: "memory"); break;
        case 24: asm volatile("s_waitcnt vmcnt(24)" ::: "memory"); break;
        case 25: asm volatile("s_waitcnt vmcnt(25)" ::: "memory"); break;
        case 26: asm volatile("s_waitcnt vmcnt(26)" ::: "memory"); break;
        case 27: asm volatile("s_waitcnt vmcnt(27)" ::: "memory"); break;
        case 28: asm volatile("s_waitcnt vmcnt(28)" ::: "memory"); break;
        case 29: asm volatile("s_waitcnt vmcnt(29)" ::: "memory"); break;
        case 30: asm volatile("s_waitcnt vmcnt(30)" ::: "memory"); break;
        default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    }
}

// Scheduling hint for the code just before it: alternate one MFMA with one LDS read, N times,
// so the fragment reads of the next K half spread over the MFMAs of the current one instead
// of bunching at the start (mask 0x008 = MFMA, 0x100 = DS read).
template <int N>
__device__ __forceinline__ void interleave_reads_with_mfmas() {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
}

// s_waitcnt lgkmcnt(0) that stays after the MFMAs issued before it: an inline-asm wait does
// not order MFMAs (they touch no memory), so without the scheduling barrier the compiler may
// hoist it above them and stall on the LDS reads with the matrix pipe idle.
// Scalar loads share the LDS wait counter but complete out of order, so while the compiler
// counts one as pending it can wait for an LDS read only with lgkmcnt(0), i.e. for every LDS
// read in flight.  A wait it can see (not inline assembly) before a K loop settles the scalar
// loads issued outside it, and the loop's waits then cover only the reads an MFMA needs.
__device__ __forceinline__ void settle_scalar_loads() {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left at their maxima
}

__device__ __forceinline__ void wait_lds_after_mfmas() {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Workgroup barrier WITHOUT the memory fence of __syncthreads(): that fence waits for every
// outstanding global load (vmcnt(0)), which would also wait for the direct-to-LDS loads of
// the stages still in flight.  Visibility is handled explicitly instead: each wave waits
// (wait_vmcnt) for the loads of the stage about to be read, and its own LDS reads of the
// stage about to be overwritten have completed because the MFMAs consumed them.
__device__ __forceinline__ void stage_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------------------
// Kernel arguments
// ---------------------------------------------------------------------------------------

// One output matrix of a launch: one (prime, part) of a CP-MM, or the single output of a
// Mod-PP-MM.  Global column tiles [tile_begin, tile_begin + tiles) belong to it.
struct Seg {
    uint64_t *C;        // output, row stride ldc
    const uint64_t *X;  // FP64 form: right operand (k x n, row stride ldx); INT8: unused
    int64_t ldc, ldx;
    int64_t n;          // valid columns
    uint64_t q;
    double qinv;        // 1.0 / q rounded to double
    uint64_t wmod;      // 2^limb_bits mod q  (Horner multiplier)
    uint64_t wshoup;    // floor(wmod * 2^64 / q)
    int32_t tile_begin; // first global column tile
    int32_t tiles;      // column tiles of this segment
};

struct GemmArgs {
    // INT8 form: digit planes in the tile-major layout described above.
    const int8_t *Pd;
    const int8_t *Xd;
    // FP64 form: the plaintext / left operand read directly (signed int64 or residues).
    const int64_t *P;
    int64_t ldp;
    int64_t m;           // valid rows
    int64_t k;           // valid K (FP64 form masks loads beyond it)
    int32_t kblocks;     // K blocks (stages) of the launch
    int32_t kfold;       // stages accumulated before a fold (>= kblocks: never)
    int32_t tiles_m, tiles_n;
    int32_t group_m;     // row tiles per raster group
    int32_t n_xcd;       // XCDs the hardware deals workgroups to round-robin
    int32_t limb_bits;   // FP64 form: bits per limb
    int32_t nseg;
    Seg seg[kMaxSegs];
};

// One job of a batched digit split: a whole matrix of one problem, split into the tile-major
// workspace; the job owns workgroups [wg_start, wg_start + tiles * kblocks).
struct SplitJob {
    int64_t wg_start;
    const int64_t *P;   // plaintext side (rows_side = 1): rows x k, row stride ld
    const uint64_t *X;  // ciphertext side (rows_side = 0): k x cols, row stride ld
    int64_t ld, rows, cols, k;
    int32_t kblocks, R, rows_side, pad;
    int8_t *out;
};

// A problem of a batch: its digit workspaces, tiles and output segments (seg0 .. seg0+nseg).
struct BatchProb {
    int64_t item_start;  // first work item (tile) of the problem in the batch's work list
    const int8_t *Pd;
    const int8_t *Xd;
    int64_t m;
    int32_t kblocks, tiles_m, tiles_n, cls, seg0, nseg;
};

struct BatchSeg {
    uint64_t *C;
    int64_t ldc, n;
    uint64_t q;
    double qinv;
    int32_t tile_begin, pad;
};

// The work list is cut into n_chunks contiguous chunks of about equal cost, one per XCD;
// chunk x is [chunk_begin[x], chunk_begin[x+1]) and counters[x] hands out its items.
constexpr int kMaxChunks = 16;
struct BatchArgs {
    const BatchProb *probs;
    const BatchSeg *segs;
    unsigned int *counters;  // kMaxChunks counters, zeroed by a reset kernel before each launch
    int64_t total_items;
    int64_t chunk_begin[kMaxChunks + 1];
    int32_t nprob, kfold, group_m, n_chunks;
};

// Constants of a rescale by the last of L primes: q mod q_l and q^{-1} mod q_l (Shoup form).
constexpr int kMaxRescalePrimes = 64;
struct RescaleConsts {
    int32_t L, pad;
    uint64_t q[kMaxRescalePrimes];
    uint64_t q_mod[kMaxRescalePrimes];
    uint64_t qinv[kMaxRescalePrimes];
    uint64_t qinv_shoup[kMaxRescalePrimes];
};

// Maps a workgroup id to (row tile, column tile).  Workgroups are dealt to the XCDs
// round-robin, so ids w, w+n_xcd, ... share an XCD and its L2.  The remap gives every XCD a
// contiguous run of logical tiles, and the raster walks group_m row tiles column by column
// within each group, so co-resident workgroups of one XCD share plaintext row panels and
// ciphertext column panels in that L2.
__device__ __forceinline__ void map_tile(int w, int total, int n_xcd, int tiles_m, int tiles_n,
                                         int group_m, int &rb, int &cb) {
    int t = w;
    if (n_xcd > 1) {
        const int per = total / n_xcd, rem = total % n_xcd;
        const int x = w % n_xcd, local = w / n_xcd;
        t = (x < rem) ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
    }
    const int span = group_m * tiles_n;
    const int g = t / span;
    const int first = g * group_m;
    const int gm = min(group_m, tiles_m - first);
    const int in = t - g * span;
    rb = first + in % gm;
    cb = in / gm;
}

__device__ __forceinline__ int find_seg(const GemmArgs &a, int cb) {
    int s = 0;
#pragma unroll 1
    for (int i = 1; i < a.nseg; ++i)
        if (cb >= a.seg[i].tile_begin) s = i;
    return s;
}

}  // namespace hlb
