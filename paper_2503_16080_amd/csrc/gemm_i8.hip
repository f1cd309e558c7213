// gemm_i8.hip -- INT8-digit form of the exact Mod-PP-MM on gfx950 matrix cores.
//
// Strategy 1 of Section 6.1 (Lemma le:strategy1, Eq decomp) with base K = 256 and balanced
// signed digits: both operands are split into int8 digit planes, every digit-plane pair
// P_i * X_j is multiplied exactly on v_mfma_i32_32x32x32_i8 and accumulated into the int32
// accumulator of its shift s = i + j, and the epilogue recombines sum_s c_s 256^s and
// reduces it modulo q (Horner, one reduction per shift) into the canonical residue.
//
// Exactness: a shift collects at most `pairs` digit products of magnitude <= 128*128 per K
// element, so |c_s| <= pairs * kchunk * 2^14 < 2^31 for the K chunk the host plans; longer
// K is cut into chunks whose partial results are folded into a 64-bit residue.
//
// Contents: digit-split kernels (single problem and batched), the persistent kernel of a
// batch, and the launchers of the exact grid kernel (its tile body is in i8_tile.hpp).
#include "common.hpp"
#include "i8_tile.hpp"
#include "launch.hpp"

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
constexpr int kSplitLds = 7 * 128 * kSplitRowPad;

// Keeps the compiler from turning a load whose value a later select may discard back into
// a conditional load (a branch per element, each waiting for its load): the empty asm
// consumes every loaded value unconditionally, after all the loads have been issued.
template <int N>
__device__ __forceinline__ void pin_loaded(uint64_t (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]));
}

template <int D>
__device__ __forceinline__ void digits4(const uint64_t (&x)[4], uint32_t (&out)[D]) {
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
template <int D, int R>
__device__ __forceinline__ void split_rows_tile(const int64_t *__restrict__ P, int64_t ldp, int64_t m,
                                                int64_t k, int kblocks, int rb, int kb, int8_t *out,
                                                uint8_t *lds) {
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
        digits4<D>(x[it], d);
#pragma unroll
        for (int j = 0; j < D; ++j) *(uint32_t *)(lds + (j * R + r) * kSplitRowPad + quad * 4) = d[j];
    }
    __syncthreads();
    split_stage2<D, R>(lds, out + ((int64_t)rb * kblocks + kb) * (D * R * kBK8));
}

// One (column tile cb, k block kb) of the ciphertext side: columns of X (transposed).  Each
// lane owns one column and loads 4 consecutive rows at a time, so lanes with consecutive
// columns read consecutive addresses; loads are issued first as above.
template <int D, int R>
__device__ __forceinline__ void split_cols_tile(const uint64_t *__restrict__ X, int64_t ldx, int64_t k,
                                                int64_t n, int kblocks, int cb, int kb, int8_t *out,
                                                uint8_t *lds) {
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
        digits4<D>(x[it], d);
#pragma unroll
        for (int j = 0; j < D; ++j) *(uint32_t *)(lds + (j * R + c) * kSplitRowPad + qd * 4) = d[j];
    }
    __syncthreads();
    split_stage2<D, R>(lds, out + ((int64_t)cb * kblocks + kb) * (D * R * kBK8));
}

template <int D, int R>
__global__ __launch_bounds__(kThreads) void split_rows_i8(const int64_t *__restrict__ P, int64_t ldp,
                                                          int64_t m, int64_t k, int kblocks,
                                                          int8_t *__restrict__ out) {
    __shared__ uint8_t lds[D * R * kSplitRowPad];
    split_rows_tile<D, R>(P, ldp, m, k, kblocks, blockIdx.x / kblocks, blockIdx.x % kblocks, out, lds);
}

template <int D, int R>
__global__ __launch_bounds__(kThreads) void split_cols_i8(const uint64_t *__restrict__ X, int64_t ldx,
                                                          int64_t k, int64_t n, int kblocks,
                                                          int8_t *__restrict__ out) {
    __shared__ uint8_t lds[D * R * kSplitRowPad];
    split_cols_tile<D, R>(X, ldx, k, n, kblocks, blockIdx.x / kblocks, blockIdx.x % kblocks, out, lds);
}

// Batched splits: one launch covers every job of a batch; workgroup w finds its job in a
// host-built workgroup -> job map.
template <int D>
__global__ __launch_bounds__(kThreads) void split_batch_i8(const SplitJob *__restrict__ jobs,
                                                           const int32_t *__restrict__ wg_job) {
    __shared__ uint8_t lds[kSplitLds];
    const int64_t w = blockIdx.x;
    const int ji = wg_job[w];  // one load instead of a search over the jobs
    const SplitJob &j = jobs[ji];
    const int64_t local = w - j.wg_start;
    const int tile = (int)(local / j.kblocks), kb = (int)(local % j.kblocks);
    if (j.rows_side) {
        if (j.R == 128) split_rows_tile<D, 128>(j.P, j.ld, j.rows, j.k, j.kblocks, tile, kb, j.out, lds);
        else split_rows_tile<D, 64>(j.P, j.ld, j.rows, j.k, j.kblocks, tile, kb, j.out, lds);
    } else {
        if (j.R == 128) split_cols_tile<D, 128>(j.X, j.ld, j.k, j.cols, j.kblocks, tile, kb, j.out, lds);
        else split_cols_tile<D, 64>(j.X, j.ld, j.k, j.cols, j.kblocks, tile, kb, j.out, lds);
    }
}

// ---------------------------------------------------------------------------------------
// Persistent batch kernel: a fixed grid of workgroups (one per CU) pulls output tiles from
// a work list ordered by the host (largest K first).  The list is cut into one contiguous
// chunk of about equal cost per XCD; workgroups are dealt to XCDs round-robin, so workgroup
// w serves chunk w % n_chunks first, and neighbouring tiles (which share plaintext and
// ciphertext panels) stay in one XCD's L2.  A workgroup whose chunk is exhausted moves on
// to the next chunk (work stealing) and exits after finding all n_chunks exhausted.  Each
// item maps to a problem by binary search over the problems' first work-item indices, then
// to a tile of that problem in its own tile class.
// ---------------------------------------------------------------------------------------
template <int DP, int DX, bool FOLD>
__global__ __launch_bounds__(256 * 2, 1) void gemm_i8_batch_kernel(const BatchArgs args) {
    constexpr int L0 = Class0<DP, DX>::LDS, L1 = Class1<DP, DX>::LDS;
    __shared__ __attribute__((aligned(16))) int8_t lds[L0 > L1 ? L0 : L1];
    __shared__ int64_t item;
    int chunk = blockIdx.x % args.n_chunks;
    int exhausted = 0;
    while (exhausted < args.n_chunks) {
        if (threadIdx.x == 0) {
            const int64_t t = args.chunk_begin[chunk] + (int64_t)atomicAdd(&args.counters[chunk], 1u);
            item = t < args.chunk_begin[chunk + 1] ? t : -1;
        }
        __syncthreads();
        const int64_t t = item;
        __syncthreads();  // everyone has read `item` before thread 0 overwrites it
        if (t < 0) {
            chunk = chunk + 1 == args.n_chunks ? 0 : chunk + 1;
            ++exhausted;
            continue;
        }
        exhausted = 0;
        int lo = 0, hi = args.nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (args.probs[mid].item_start <= t) lo = mid;
            else hi = mid - 1;
        }
        const BatchProb &p = args.probs[lo];
        const int local = (int)(t - p.item_start);
        // raster inside the problem: group_m row tiles walked column by column
        const int span = args.group_m * p.tiles_n;
        const int g = local / span, first = g * args.group_m;
        const int gm = min(args.group_m, p.tiles_m - first);
        const int in = local - g * span;
        const int rb = first + in % gm, cb = in / gm;
        int s = p.seg0;
        for (int i = p.seg0 + 1; i < p.seg0 + p.nseg; ++i)
            if (cb >= args.segs[i].tile_begin) s = i;
        const BatchSeg &sg = args.segs[s];
        TileJob job;
        job.KB = p.kblocks;
        job.kfold = args.kfold;
        job.m = p.m;
        job.n = sg.n;
        job.C = sg.C;
        job.ldc = sg.ldc;
        job.q = sg.q;
        job.qinv = sg.qinv;
        if (p.cls == 0) {
            using T = Class0<DP, DX>;
            job.gP = p.Pd + (int64_t)rb * p.kblocks * T::P_TILE;
            job.gX = p.Xd + (int64_t)cb * p.kblocks * T::X_TILE;
            job.row0 = (int64_t)rb * T::BM;
            job.col0 = (int64_t)(cb - sg.tile_begin) * T::BN;
            run_tile<T, FOLD>(job, lds);
        } else {
            using T = Class1<DP, DX>;
            job.gP = p.Pd + (int64_t)rb * p.kblocks * T::P_TILE;
            job.gX = p.Xd + (int64_t)cb * p.kblocks * T::X_TILE;
            job.row0 = (int64_t)rb * T::BM;
            job.col0 = (int64_t)(cb - sg.tile_begin) * T::BN;
            run_tile<T, FOLD>(job, lds);
        }
    }
}

__global__ void reset_counter_kernel(unsigned int *counters) {
    if (threadIdx.x < kMaxChunks && blockIdx.x == 0) counters[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
template <int D, int R>
static hipError_t launch_split_rows_t(const int64_t *P, int64_t ldp, int64_t m, int64_t k,
                                      int tiles, int kblocks, int8_t *out, hipStream_t s) {
    hipLaunchKernelGGL((split_rows_i8<D, R>), dim3(tiles * kblocks), dim3(kThreads), 0, s, P, ldp,
                       m, k, kblocks, out);
    return hipGetLastError();
}

template <int D, int R>
static hipError_t launch_split_cols_t(const uint64_t *X, int64_t ldx, int64_t k, int64_t n,
                                      int tiles, int kblocks, int8_t *out, hipStream_t s) {
    hipLaunchKernelGGL((split_cols_i8<D, R>), dim3(tiles * kblocks), dim3(kThreads), 0, s, X, ldx,
                       k, n, kblocks, out);
    return hipGetLastError();
}

hipError_t launch_split_rows_i8(int D, int R, const int64_t *P, int64_t ldp, int64_t m, int64_t k,
                                int tiles, int kblocks, int8_t *out, hipStream_t s) {
    if (tiles <= 0 || kblocks <= 0) return hipSuccess;
    if (R == 128 && D == 3) return launch_split_rows_t<3, 128>(P, ldp, m, k, tiles, kblocks, out, s);
    if (R == 64 && D == 3) return launch_split_rows_t<3, 64>(P, ldp, m, k, tiles, kblocks, out, s);
    if (R == 64 && D == 7) return launch_split_rows_t<7, 64>(P, ldp, m, k, tiles, kblocks, out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_split_cols_i8(int D, int R, const uint64_t *X, int64_t ldx, int64_t k, int64_t n,
                                int tiles, int kblocks, int8_t *out, hipStream_t s) {
    if (tiles <= 0 || kblocks <= 0) return hipSuccess;
    if (R == 64 && D == 7) return launch_split_cols_t<7, 64>(X, ldx, k, n, tiles, kblocks, out, s);
    if (R == 64 && D == 6) return launch_split_cols_t<6, 64>(X, ldx, k, n, tiles, kblocks, out, s);
    if (R == 128 && D == 7) return launch_split_cols_t<7, 128>(X, ldx, k, n, tiles, kblocks, out, s);
    if (R == 128 && D == 6) return launch_split_cols_t<6, 128>(X, ldx, k, n, tiles, kblocks, out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_split_batch_i8(int D, const SplitJob *jobs, const int32_t *wg_job, int64_t total_wgs,
                                 hipStream_t s) {
    if (total_wgs <= 0) return hipSuccess;
    if (total_wgs > INT32_MAX) return hipErrorInvalidValue;
    if (D == 3) hipLaunchKernelGGL(split_batch_i8<3>, dim3((unsigned)total_wgs), dim3(kThreads), 0, s, jobs, wg_job);
    else if (D == 6) hipLaunchKernelGGL(split_batch_i8<6>, dim3((unsigned)total_wgs), dim3(kThreads), 0, s, jobs, wg_job);
    else if (D == 7) hipLaunchKernelGGL(split_batch_i8<7>, dim3((unsigned)total_wgs), dim3(kThreads), 0, s, jobs, wg_job);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

I8Shape i8_shape(int dp, int dx, int cls) {
    if (dp == 3 && (dx == 7 || dx == 6)) return cls == 1 ? I8Shape{3, dx, 64, 128} : I8Shape{3, dx, 128, 64};
    if (dp == 7 && dx == 7) return {7, 7, 64, 64};
    return {0, 0, 0, 0};
}

hipError_t launch_gemm_i8(int dp, int dx, int cls, const GemmArgs &a, hipStream_t s) {
    if (dp == 3 && dx == 7) return cls == 1 ? launch_gemm_fold<Class1<3, 7>>(a, s) : launch_gemm_fold<Class0<3, 7>>(a, s);
    if (dp == 3 && dx == 6) return cls == 1 ? launch_gemm_fold<Class1<3, 6>>(a, s) : launch_gemm_fold<Class0<3, 6>>(a, s);
    if (dp == 7 && dx == 7) return launch_gemm_fold<I8Tile<7, 7, 2, 2>>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_reset_counter(unsigned int *counter, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_gemm_i8_batch(int dp, int dx, bool fold, const BatchArgs &a, int grid, hipStream_t s) {
    if (grid <= 0 || a.total_items <= 0) return hipSuccess;
#define HLB_BATCH(DP_, DX_)                                                                         \
    if (dp == DP_ && dx == DX_) {                                                                   \
        if (fold) hipLaunchKernelGGL((gemm_i8_batch_kernel<DP_, DX_, true>), dim3(grid), dim3(512), 0, s, a);  \
        else hipLaunchKernelGGL((gemm_i8_batch_kernel<DP_, DX_, false>), dim3(grid), dim3(512), 0, s, a);      \
        return hipGetLastError();                                                                   \
    }
    HLB_BATCH(3, 7)
    HLB_BATCH(3, 6)
#undef HLB_BATCH
    return hipErrorInvalidValue;
}

}  // namespace hlb
