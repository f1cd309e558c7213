// gemm_f64.hip -- FP64-limb form of the exact Mod-PP-MM on gfx950 matrix cores.
//
// This is Strategy 1 of Section 6.1 as the paper states it (Lemma le:strategy1, Eq decomp):
// the operands are chopped into limbs of w bits, every limb product P_i * X_j is computed
// on the FP64 matrix cores (v_mfma_f64_16x16x4_f64), where all partial sums are integers of
// magnitude < 2^53 and hence exact, and the limb products are recombined over the integers
// and reduced modulo q.  The right operand is split into NX unsigned limbs; the plaintext
// into NP sign-magnitude limbs (the paper's digits "of the sign of r"), NP = 1 being the
// paper's choice k2 = 1 for a low-precision plaintext (Section 6.3).  Products sharing a
// shift s = i + j share one FP64 accumulator; the host sizes w and the K chunk so that
// pairs * kchunk * max|P_i| * max|X_j| < 2^53, folding longer K into 64-bit residues.
//
// This kernel needs no workspace: the limb split happens on the way from global memory into
// LDS (register-staged).  It serves every limb count; the one-plaintext-limb plans of the
// CP-MM run by default on the plane kernel of gemm_f64_planes.hip instead.
//
// TRUNC = true is Strategy 2 of Section 6.1 instead: one FP64 product of the operands
// rounded to doubles (the plaintext as a signed integer, the residues in their centred
// representatives in (-q/2, q/2]), whose integer-valued result is then reduced modulo q.
// Not exact: the accumulation rounds once the partial sums pass 2^53.
#include "common.hpp"
#include "launch.hpp"

namespace hlb {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int NP_, int NX_>
struct F64Tile {
    static constexpr int NP = NP_, NX = NX_, NS = NP + NX - 1;
    static constexpr int BM = 64, BN = 64, BK = kBK64;
    // LDS doubles per stage: P limbs [NP][BK][BM] and X limbs [NX][BK][BN]
    static constexpr int P_ELEMS = NP * BK * BM, X_ELEMS = NX * BK * BN;
    static constexpr int STAGE = P_ELEMS + X_ELEMS;
};

template <class T, bool FOLD, bool TRUNC = false>
__global__ __launch_bounds__(kThreads, 1) void gemm_f64_kernel(const GemmArgs args) {
    static_assert(!TRUNC || (T::NP == 1 && T::NX == 1 && !FOLD), "truncation: one limb each, no fold");
    __shared__ __attribute__((aligned(16))) double lds[2 * T::STAGE];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int total = args.tiles_m * args.tiles_n;
    int rb, cb;
    map_tile(blockIdx.x, total, args.n_xcd, args.tiles_m, args.tiles_n, args.group_m, rb, cb);

    const int si = find_seg(args, cb);
    const Seg &sg = args.seg[si];
    const uint64_t q = sg.q;
    const double qd = (double)q, qinv = sg.qinv;
    const int w = args.limb_bits;
    const uint64_t mask = ((uint64_t)1 << w) - 1;

    const int64_t m0 = (int64_t)rb * T::BM;
    const int64_t n0 = (int64_t)(cb - sg.tile_begin) * T::BN;
    const int64_t K = args.k;

    v4d acc[2][2][T::NS];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int s = 0; s < T::NS; ++s) acc[a][b][s] = v4d{0.0, 0.0, 0.0, 0.0};
    uint64_t part[FOLD ? 2 : 1][FOLD ? 2 : 1][FOLD ? 4 : 1];
    if constexpr (FOLD) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) part[a][b][i] = 0;
    }

    // per-thread load coordinates: P tile 64 x 16 (row pr, 4 K from pk), X tile 16 x 64
    const int pr = tid >> 2, pk = (tid & 3) * 4;
    const int xk = tid >> 4, xn = (tid & 15) * 4;
    int64_t rp[4];
    uint64_t rx[4];
    auto gload = [&](int kb) {
        // loads from clamped in-bounds addresses, then selects
        const int64_t k0 = (int64_t)kb * T::BK;
        const int64_t row = m0 + pr;
        const int64_t rowc = row < args.m ? row : args.m - 1;
        const int64_t kr = k0 + xk;
        const int64_t krc = kr < K ? kr : K - 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            rp[e] = args.P[rowc * args.ldp + (k0 + pk + e < K ? k0 + pk + e : K - 1)];
            const int64_t col = n0 + xn + e;
            rx[e] = sg.X[krc * sg.ldx + (col < sg.n ? col : sg.n - 1)];
        }
        // the empty asm consumes every loaded value unconditionally, so the masks below
        // stay selects instead of becoming conditional loads (a branch and a wait each)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            asm volatile("" : "+v"(rp[e]));
            asm volatile("" : "+v"(rx[e]));
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            rp[e] = (row < args.m && k0 + pk + e < K) ? rp[e] : 0;
            rx[e] = (kr < K && n0 + xn + e < sg.n) ? rx[e] : 0;
        }
    };
    auto lstore = [&](int buf) {
        double *lp = lds + buf * T::STAGE;
        double *lx = lp + T::P_ELEMS;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t v = rp[e];
            if constexpr (T::NP == 1) {
                lp[(pk + e) * T::BM + pr] = (double)v;
            } else {
                const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
                const double sgn = v < 0 ? -1.0 : 1.0;
#pragma unroll
                for (int i = 0; i < T::NP; ++i)
                    lp[(i * T::BK + pk + e) * T::BM + pr] = sgn * (double)((mag >> (w * i)) & mask);
            }
        }
        if constexpr (TRUNC) {
            // centred representative: x - q when 2x > q
            double c[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                c[e] = (double)(2 * rx[e] > q ? (int64_t)rx[e] - (int64_t)q : (int64_t)rx[e]);
            double2 *dst = (double2 *)(lx + xk * T::BN + xn);
            dst[0] = double2{c[0], c[1]};
            dst[1] = double2{c[2], c[3]};
            return;
        }
#pragma unroll
        for (int j = 0; j < T::NX; ++j) {
            double2 lo, hi;
            lo.x = (double)((rx[0] >> (w * j)) & mask);
            lo.y = (double)((rx[1] >> (w * j)) & mask);
            hi.x = (double)((rx[2] >> (w * j)) & mask);
            hi.y = (double)((rx[3] >> (w * j)) & mask);
            double2 *dst = (double2 *)(lx + (j * T::BK + xk) * T::BN + xn);
            dst[0] = lo;
            dst[1] = hi;
        }
    };
    auto compute = [&](int buf) {
        const double *lp = lds + buf * T::STAGE;
        const double *lx = lp + T::P_ELEMS;
#pragma unroll
        for (int kk = 0; kk < T::BK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double a[2][T::NP], b[2][T::NX];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int i = 0; i < T::NP; ++i)
                    a[mb][i] = lp[(i * T::BK + kr) * T::BM + wm * 32 + mb * 16 + (lane & 15)];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int j = 0; j < T::NX; ++j)
                    b[nb][j] = lx[(j * T::BK + kr) * T::BN + wn * 32 + nb * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < T::NP; ++i)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                        for (int j = 0; j < T::NX; ++j)
                            acc[mb][nb][i + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                a[mb][i], b[nb][j], acc[mb][nb][i + j], 0, 0, 0);
        }
    };
    // sum_s c_s 2^{w s} mod q by Horner from the top shift, every c_s an exact integer
    auto recombine = [&](int a, int b, int i) -> uint64_t {
        uint64_t r = reduce_fp(acc[a][b][T::NS - 1][i], q, qd, qinv);
#pragma unroll
        for (int s = T::NS - 2; s >= 0; --s)
            r = addmod(mulmod_shoup(r, sg.wmod, sg.wshoup, q), reduce_fp(acc[a][b][s][i], q, qd, qinv), q);
        return r;
    };
    auto fold = [&]() {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) part[a][b][i] = addmod(part[a][b][i], recombine(a, b, i), q);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int s = 0; s < T::NS; ++s) acc[a][b][s] = v4d{0.0, 0.0, 0.0, 0.0};
    };

    const int KB = args.kblocks;
    gload(0);
    lstore(0);
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < KB; ++kb) {
        const int cur = kb & 1;
        if (kb + 1 < KB) gload(kb + 1);
        compute(cur);
        if (kb + 1 < KB) lstore(cur ^ 1);
        if constexpr (FOLD) {
            if ((kb + 1) % args.kfold == 0 && kb + 1 < KB) fold();
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // 16x16 FP64 accumulator layout: column = lane % 16, row = 4 i + lane / 16
                const int64_t row = m0 + wm * 32 + a * 16 + 4 * i + (lane >> 4);
                const int64_t col = n0 + wn * 32 + b * 16 + (lane & 15);
                uint64_t v;
                if constexpr (TRUNC) v = reduce_fp(acc[a][b][0][i], q, qd, qinv);  // |acc| < q 2^51
                else v = recombine(a, b, i);
                if constexpr (FOLD) v = addmod(v, part[a][b][i], q);
                if (row < args.m && col < sg.n) sg.C[row * sg.ldc + col] = v;
            }
}

template <class T, bool FOLD>
static hipError_t launch_t(const GemmArgs &a, hipStream_t s) {
    const int grid = a.tiles_m * a.tiles_n;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_f64_kernel<T, FOLD>), dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <class T>
static hipError_t launch_fold(const GemmArgs &a, hipStream_t s) {
    return a.kfold < a.kblocks ? launch_t<T, true>(a, s) : launch_t<T, false>(a, s);
}

bool f64_supported(int np, int nx) {
    return (np == 1 && (nx == 3 || nx == 4)) || (np == 3 && nx == 3) || (np == 4 && nx == 4);
}

hipError_t launch_gemm_f64_trunc(const GemmArgs &a, hipStream_t s) {
    const int grid = a.tiles_m * a.tiles_n;
    if (grid <= 0) return hipSuccess;
    if (a.kfold < a.kblocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_f64_kernel<F64Tile<1, 1>, false, true>), dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm_f64(int np, int nx, const GemmArgs &a, hipStream_t s) {
    if (np == 1 && nx == 3) return launch_fold<F64Tile<1, 3>>(a, s);
    if (np == 1 && nx == 4) return launch_fold<F64Tile<1, 4>>(a, s);
    if (np == 3 && nx == 3) return launch_fold<F64Tile<3, 3>>(a, s);
    if (np == 4 && nx == 4) return launch_fold<F64Tile<4, 4>>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace hlb
