// crt_gemm_batch.hip -- the INT8 products of a multimodular (CRT) batch: every (problem,
// modulus, output tile) of a batch of CP-MMs in one launch, over the residue planes written
// by the batched split (crt.hip).  The tile itself is in crt_tile.hpp; the host resolves
// every tile to its operands (batch.hip).
#include "common.hpp"
#include "crt.hpp"
#include "crt_jobs.hpp"
#include "crt_tile.hpp"
#include "launch.hpp"

#include <algorithm>

namespace hlb {

// A batch of problems in one persistent launch of `workers` workgroups (one per CU when the
// batch has that many tiles).  Workgroups are dealt to the XCDs round-robin, so workgroup w
// starts on run w % n_xcd, its own XCD's, and takes that run's items in order from an atomic
// counter (neighbouring items share operand panels in the XCD's L2).  When its run is
// exhausted it moves on to the next run (work stealing, which absorbs any error of the host's
// cost estimate), and it exits once it has found every run exhausted in a row.  The host has
// resolved every item to its operands, so an item starts with one descriptor load.
template <class T>
__global__ __launch_bounds__(T::THREADS, 1) void crt_gemm_batch_kernel(const CrtBatchArgs args) {
    __shared__ __attribute__((aligned(16))) int8_t lds[T::NBUF * T::STAGE];
    // the tile's pipeline fills all of LDS, so the item index passes through its first bytes
    volatile int64_t *next = (volatile int64_t *)lds;
    static_assert(T::XSUB <= kCrtItemCols, "one destination per plane tile of the batch tile");
    int run = (int)(blockIdx.x % args.n_xcd);
    int exhausted = 0;
    while (exhausted < args.n_xcd) {
        __syncthreads();  // every wave is done with the last tile's LDS
        if (threadIdx.x == 0) {
            const int64_t t = args.chunk[run] + (int64_t)atomicAdd(&args.counters[run], 1u);
            *next = t < args.chunk[run + 1] ? t : -1;
        }
        __syncthreads();
        // uniform (an LDS value is taken as per-lane otherwise): the tile's branches, loop
        // bounds and addresses stay scalar
        const int64_t t = __builtin_amdgcn_readfirstlane((int)*next);
        __syncthreads();  // every wave has read it before the tile's loads overwrite it
        if (t < 0) {
            run = run + 1 == args.n_xcd ? 0 : run + 1;
            ++exhausted;
            continue;
        }
        exhausted = 0;
        const CrtItem &it = args.items[t];  // read in place: the epilogue indexes its arrays by wave
        auto dst = [&](int bc) -> CrtBlockCol {
            const int j = bc / 4;
            if (!it.Y[j]) return {nullptr, 0};
            return {it.Y[j] + ((int64_t)it.brt * it.nbc[j] + it.bct[j] + bc % 4) * 1024, it.nbc[j] * 1024};
        };
        crt_tile<T>(lds, it.P, it.X, it.kblocks, (int64_t)args.D * kCrtSub, it.p, dst);
    }
}

// ---------------------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------------------
template <class T>
static hipError_t launch_batch_t(const CrtBatchArgs &a, int workers, hipStream_t s) {
    const int64_t grid = std::min<int64_t>(workers, a.total_items);
    hipLaunchKernelGGL(crt_gemm_batch_kernel<T>, dim3((unsigned)grid), dim3(T::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_crt_gemm_batch(int variant, const CrtBatchArgs &a, int workers, hipStream_t s) {
    if (a.total_items <= 0) return hipSuccess;
    if (a.n_xcd < 1 || a.n_xcd > kMaxChunks || a.total_items > INT32_MAX || workers < 1 || !a.counters)
        return hipErrorInvalidValue;
    if (variant == 0) return launch_batch_t<CrtNarrow>(a, workers, s);
    if (variant == 1) return launch_batch_t<CrtWide>(a, workers, s);
    if (variant == 2) return launch_batch_t<CrtWider>(a, workers, s);
    return hipErrorInvalidValue;
}

}  // namespace hlb
