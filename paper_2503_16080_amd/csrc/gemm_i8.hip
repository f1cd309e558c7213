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
#include "split.hpp"

namespace hlb {

template <int D, int R>
__global__ __launch_bounds__(kThreads) void split_rows_i8(const int64_t *__restrict__ P, int64_t ldp,
                                                          int64_t m, int64_t k, int kblocks,
                                                          int8_t *__restrict__ out) {
    __shared__ uint8_t lds[D * R * kSplitRowPad];
    split_rows_tile<D, R>(P, ldp, m, k, kblocks, blockIdx.x / kblocks, blockIdx.x % kblocks, out, lds,
                          DigitConv<D>{});
}

template <int D, int R>
__global__ __launch_bounds__(kThreads) void split_cols_i8(const uint64_t *__restrict__ X, int64_t ldx,
                                                          int64_t k, int64_t n, int kblocks,
                                                          int8_t *__restrict__ out) {
    __shared__ uint8_t lds[D * R * kSplitRowPad];
    split_cols_tile<D, R>(X, ldx, k, n, kblocks, blockIdx.x / kblocks, blockIdx.x % kblocks, out, lds,
                          DigitConv<D>{});
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
        if (j.R == 128) split_rows_tile<D, 128>(j.P, j.ld, j.rows, j.k, j.kblocks, tile, kb, j.out, lds, DigitConv<D>{});
        else split_rows_tile<D, 64>(j.P, j.ld, j.rows, j.k, j.kblocks, tile, kb, j.out, lds, DigitConv<D>{});
    } else {
        if (j.R == 128) split_cols_tile<D, 128>(j.X, j.ld, j.k, j.cols, j.kblocks, tile, kb, j.out, lds, DigitConv<D>{});
        else split_cols_tile<D, 64>(j.X, j.ld, j.k, j.cols, j.kblocks, tile, kb, j.out, lds, DigitConv<D>{});
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
