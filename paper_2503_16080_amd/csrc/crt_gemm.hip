// crt_gemm.hip -- the INT8 products of one multimodular (CRT) call: every (modulus, output
// tile) of the call's products in one launch, over the residue planes written by the splits
// (crt.hip).  The tile itself, and the stream of tiles a persistent workgroup runs, are in
// crt_tile.hpp.
#include "common.hpp"
#include "crt.hpp"
#include "crt_tile.hpp"
#include "launch.hpp"

#include <algorithm>

namespace hlb {

// Where tile t of a launch reads and writes.  The D moduli stack as D row bands of one
// (D tiles_m) x tiles_n grid of output tiles, numbered in raster groups of group_m row tiles;
// each XCD takes a contiguous share of that numbering (map_tile).
//
// The output matrices of a launch lie side by side in 128-column plane tiles, so a GEMM tile
// may straddle two of them (and the last may run past the end): each 32-column block of the
// tile finds its matrix, and blocks past the last one are not stored.
template <class T>
struct CrtCallTiles {
    const CrtGemmArgs &a;
    int64_t plane_stride, tile_stride;

    __device__ explicit CrtCallTiles(const CrtGemmArgs &args) : a(args) {
        plane_stride = (int64_t)a.D * kCrtSub;  // bytes of one k block of a 128-wide tile
        tile_stride = (int64_t)a.kblocks * plane_stride;
    }
    // logical tile t of the raster (already placed on its XCD)
    __device__ CrtRef ref(int t) const {
        int rbv, cb;
        map_tile(t, 0, 1, a.D * a.tiles_m, a.tiles_n, a.group_m, rbv, cb);
        // integer division runs on the vector unit: bring the (uniform) results back to
        // scalar registers
        rbv = __builtin_amdgcn_readfirstlane(rbv);
        cb = __builtin_amdgcn_readfirstlane(cb);
        const int mi = __builtin_amdgcn_readfirstlane(rbv / a.tiles_m), rb = rbv - mi * a.tiles_m;
        CrtRef r;
        r.gP = a.Pd + (int64_t)(2 * rb) * tile_stride + (int64_t)mi * kCrtSub;
        r.gX = a.Xd + (int64_t)cb * T::XSUB * tile_stride + (int64_t)mi * kCrtSub;
        r.KB = a.kblocks;
        r.p = kCrtModuli[mi];
        r.c0 = mi;
        r.c1 = rb;
        r.c2 = cb;
        return r;
    }
    __device__ CrtBlockCol dst(const CrtRef &r, int bc) const {
        const int64_t pt = r.c2 * T::XSUB + bc / 4;
#pragma unroll 1
        for (int i = 0; i < a.nseg; ++i) {
            const CrtSeg &sg = a.seg[i];
            if (pt >= sg.tile_begin && pt < sg.tile_begin + sg.tiles)
                return {sg.Y + r.c0 * sg.plane + (r.c1 * (kCrtBM / 32) * sg.nbc + (pt - sg.tile_begin) * 4 + bc % 4) * 1024,
                        sg.nbc * 1024};
        }
        return {nullptr, 0};
    }
};

// The tile queue of a persistent launch: XCD x owns a contiguous run of the raster (the
// partition of map_tile) with its own counter; a workgroup takes tiles from its XCD's run
// (workgroups are dealt to the XCDs round-robin) and, once that is exhausted, from the next
// runs in turn.  Taking tiles as workgroups free up, rather than in a fixed order, keeps the
// tiles an XCD runs at one time neighbours in the raster and in step along K, which is what
// lets them share their operand stages in the XCD's L2.
template <class T>
struct CrtCallQueue : CrtCallTiles<T> {
    int run, exhausted, per, rem;

    __device__ explicit CrtCallQueue(const CrtGemmArgs &args) : CrtCallTiles<T>(args) {
        const int total = args.D * args.tiles_m * args.tiles_n;
        run = blockIdx.x % args.n_xcd;
        exhausted = 0;
        per = total / args.n_xcd;
        rem = total % args.n_xcd;
    }
    __device__ int begin(int x) const { return x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per; }
    __device__ uint32_t claim() { return atomicAdd(&this->a.counters[run], 1u); }
    __device__ int resolve(uint32_t c) {
#pragma unroll 1
        while (true) {
            const int b = begin(run), e = begin(run + 1);
            if ((int64_t)b + c < e) {
                exhausted = 0;
                return b + (int)c;
            }
            if (++exhausted >= this->a.n_xcd) return -1;
            run = run + 1 == this->a.n_xcd ? 0 : run + 1;
            c = atomicAdd(&this->a.counters[run], 1u);
        }
    }
};

// One tile per workgroup.
template <class T>
__global__ __launch_bounds__(T::THREADS, 1) void crt_gemm_kernel(const CrtGemmArgs args) {
    __shared__ __attribute__((aligned(16))) int8_t lds[T::NBUF * T::STAGE];
    const CrtCallTiles<T> tiles(args);
    const int total = args.D * args.tiles_m * args.tiles_n;
    int rbv, cb;
    map_tile(blockIdx.x, total, args.n_xcd, 1, total, 1, rbv, cb);  // the XCD placement only
    const CrtRef r = tiles.ref(cb);
    crt_tile<T>(lds, r.gP, r.gX, r.KB, tiles.plane_stride, r.p, [&](int bc) { return tiles.dst(r, bc); });
}

// One persistent workgroup per CU over the tile queue.
template <class T>
__global__ __launch_bounds__(T::THREADS, 1) void crt_gemm_stream_kernel(const CrtGemmArgs args) {
    __shared__ __attribute__((aligned(16))) int8_t lds[T::NBUF * T::STAGE];
    CrtCallQueue<T> q(args);
    crt_tiles<T>(lds, q.plane_stride, q);
}

// ---------------------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------------------
int crt_tile_cols(int variant) { return variant == 0 ? CrtNarrow::BN : variant == 1 ? CrtWide::BN : CrtWider::BN; }

template <class T>
static hipError_t launch_crt_t(int64_t grid, const CrtGemmArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(crt_gemm_kernel<T>, dim3((unsigned)grid), dim3(T::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_crt_gemm(int variant, const CrtGemmArgs &a, int workers, hipStream_t s) {
    const int64_t total = (int64_t)a.D * a.tiles_m * a.tiles_n;
    if (total <= 0) return hipSuccess;
    if (total > INT32_MAX || a.n_xcd < 1 || a.n_xcd > kMaxChunks) return hipErrorInvalidValue;
    if (variant == 0) return launch_crt_t<CrtNarrow>(total, a, s);
    if (variant == 1) return launch_crt_t<CrtWide>(total, a, s);
    // the 256 x 384 tile: when every tile has an even K-block count of at least the ring's
    // depth, one persistent workgroup per CU streams the tile queue through the LDS ring
    // (the queue's counters zeroed beforehand); otherwise one workgroup per tile
    if (a.kblocks % 2 != 0 || a.kblocks < CrtWider::NBUF || !a.counters) return launch_crt_t<CrtWider>(total, a, s);
    hipError_t e = launch_reset_counter(a.counters, s);
    if (e != hipSuccess) return e;
    const int64_t per_xcd = std::max<int64_t>(1, std::min<int64_t>(workers / a.n_xcd, (total + a.n_xcd - 1) / a.n_xcd));
    hipLaunchKernelGGL(crt_gemm_stream_kernel<CrtWider>, dim3((unsigned)(per_xcd * a.n_xcd)), dim3(CrtWider::THREADS), 0,
                       s, a);
    return hipGetLastError();
}

}  // namespace hlb
