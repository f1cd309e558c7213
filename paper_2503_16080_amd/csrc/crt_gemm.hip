// crt_gemm.hip -- the INT8 products of one multimodular (CRT) call: every (modulus, output
// tile) of the call's products in one launch, over the residue planes written by the splits
// (crt.hip).  The tile itself is in crt_tile.hpp.
#include "common.hpp"
#include "crt.hpp"
#include "crt_tile.hpp"
#include "launch.hpp"

namespace hlb {

// The output matrices of a launch lie side by side in 128-column plane tiles, so a GEMM tile
// may straddle two of them (and the last may run past the end): each 32-column block of the
// tile finds its matrix, and blocks past the last one are not stored.
template <class T>
__global__ __launch_bounds__(T::THREADS, 1) void crt_gemm_kernel(const CrtGemmArgs args) {
    __shared__ __attribute__((aligned(16))) int8_t lds[T::NBUF * T::STAGE];
    // the D moduli stack as D row bands of one (D * tiles_m) x tiles_n grid
    const int total = args.D * args.tiles_m * args.tiles_n;
    int rbv, cb;
    map_tile(blockIdx.x, total, args.n_xcd, args.D * args.tiles_m, args.tiles_n, args.group_m, rbv, cb);
    const int mi = rbv / args.tiles_m, rb = rbv % args.tiles_m;
    const int KB = args.kblocks;
    const int64_t plane_stride = (int64_t)args.D * kCrtSub;  // bytes of one k block of a 128-wide tile
    const int64_t tile_stride = (int64_t)KB * plane_stride;
    const int64_t pt0 = (int64_t)cb * T::XSUB;  // first plane tile of this GEMM tile
    auto dst = [&](int bc) -> CrtBlockCol {
        const int64_t pt = pt0 + bc / 4;
#pragma unroll 1
        for (int i = 0; i < args.nseg; ++i) {
            const CrtSeg &sg = args.seg[i];
            if (pt >= sg.tile_begin && pt < sg.tile_begin + sg.tiles)
                return {sg.Y + (int64_t)mi * sg.plane +
                            ((int64_t)rb * (kCrtBM / 32) * sg.nbc + (pt - sg.tile_begin) * 4 + bc % 4) * 1024,
                        sg.nbc * 1024};
        }
        return {nullptr, 0};
    };
    crt_tile<T>(lds, args.Pd + (int64_t)(2 * rb) * tile_stride + (int64_t)mi * kCrtSub,
                args.Xd + pt0 * tile_stride + (int64_t)mi * kCrtSub, KB, plane_stride, kCrtModuli[mi], dst);
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

hipError_t launch_crt_gemm(int variant, const CrtGemmArgs &a, hipStream_t s) {
    const int64_t grid = (int64_t)a.D * a.tiles_m * a.tiles_n;
    if (grid <= 0) return hipSuccess;
    if (grid > INT32_MAX) return hipErrorInvalidValue;
    if (variant == 0) return launch_crt_t<CrtNarrow>(grid, a, s);
    return variant == 1 ? launch_crt_t<CrtWide>(grid, a, s) : launch_crt_t<CrtWider>(grid, a, s);
}

}  // namespace hlb
