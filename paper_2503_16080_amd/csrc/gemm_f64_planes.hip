// gemm_f64_planes.hip -- FP64 form of the CP-MM on pre-laid-out double planes.
//
// Strategy 1 of Section 6.1 with one plaintext limb (the paper's k2 = 1 for a low-precision
// plaintext, Section 6.3) and NX limbs of w bits for the residues (Lemma le:strategy1, Eq
// decomp); with TRUNC it is Strategy 2 instead: one FP64 product of the plaintext and the
// residues' centred representatives, rounded to doubles.
//
// Two passes.  The preparation kernels convert the operands once into double planes in a
// tile-major workspace, so that one LDS stage of one workgroup is one contiguous block:
//   plaintext  [row tile][k block][16 K][64 rows]            (8 KB per stage)
//   residues   [col tile][k block][limb][16 K][64 columns]   (NX * 8 KB per stage)
// with entries outside the valid m x k (or k x n) range set to zero.  The GEMM then copies
// those blocks straight into LDS (direct-to-LDS loads, several stages in flight) and its
// inner loop holds nothing but LDS fragment reads, prefetched one K step ahead, and
// v_mfma_f64_16x16x4_f64.  Products sharing a shift share an accumulator; the epilogue
// recombines and reduces them as the register-staged FP64 kernel does.
#include "common.hpp"
#include "launch.hpp"

namespace hlb {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kPlaneBM = 64, kPlaneBN = 64, kPlaneBK = kBK64;          // 64 x 64 x 16
constexpr int kPlaneBlock = kPlaneBK * kPlaneBM;                       // doubles per plane block

// ---------------------------------------------------------------------------------------
// Preparation: one workgroup per (tile, k block).
// ---------------------------------------------------------------------------------------

// Plaintext rows -> [16 K][64 rows] doubles (a transpose through LDS: loads read 4
// consecutive K of one row, stores write 4 consecutive rows of one K).
__global__ __launch_bounds__(kThreads) void prep_p_planes(const int64_t *__restrict__ P, int64_t ldp, int64_t m,
                                                          int64_t k, int kblocks, double *__restrict__ out) {
    __shared__ double t[kPlaneBK][kPlaneBM + 1];
    const int tile = blockIdx.x / kblocks, kb = blockIdx.x % kblocks;
    const int tid = threadIdx.x;
    const int r = tid >> 2, kq = (tid & 3) * 4;
    const int64_t row = (int64_t)tile * kPlaneBM + r;
    const int64_t k0 = (int64_t)kb * kPlaneBK + kq;
    const int64_t rowc = row < m ? row : m - 1;
    int64_t v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = P[rowc * ldp + (k0 + e < k ? k0 + e : k - 1)];
#pragma unroll
    for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(v[e]));  // keep the masks below selects
#pragma unroll
    for (int e = 0; e < 4; ++e) t[kq + e][r] = (row < m && k0 + e < k) ? (double)v[e] : 0.0;
    __syncthreads();
    const int kk = tid >> 4, c = (tid & 15) * 4;
    double *dst = out + ((int64_t)tile * kblocks + kb) * kPlaneBlock + kk * kPlaneBM + c;
    *(double2 *)dst = double2{t[kk][c], t[kk][c + 1]};
    *(double2 *)(dst + 2) = double2{t[kk][c + 2], t[kk][c + 3]};
}

// Residue rows -> NX limb planes [limb][16 K][64 columns] (or, with TRUNC, one plane of
// centred representatives).  Thread: one K row, 4 consecutive columns.
template <int NX, bool TRUNC>
__global__ __launch_bounds__(kThreads) void prep_x_planes(const uint64_t *__restrict__ X, int64_t ldx, int64_t k,
                                                          int64_t n, int kblocks, int w, uint64_t q,
                                                          double *__restrict__ out) {
    const int tile = blockIdx.x / kblocks, kb = blockIdx.x % kblocks;
    const int tid = threadIdx.x;
    const int kk = tid >> 4, c = (tid & 15) * 4;
    const int64_t krow = (int64_t)kb * kPlaneBK + kk;
    const int64_t col = (int64_t)tile * kPlaneBN + c;
    const int64_t kc = krow < k ? krow : k - 1;
    uint64_t x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = X[kc * ldx + (col + e < n ? col + e : n - 1)];
#pragma unroll
    for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(x[e]));
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = (krow < k && col + e < n) ? x[e] : 0;
    double *dst = out + ((int64_t)tile * kblocks + kb) * NX * kPlaneBlock + kk * kPlaneBN + c;
    const uint64_t mask = ((uint64_t)1 << w) - 1;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
        double d[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if constexpr (TRUNC) d[e] = (double)(2 * x[e] > q ? (int64_t)x[e] - (int64_t)q : (int64_t)x[e]);
            else d[e] = (double)(uint32_t)((x[e] >> (w * j)) & mask);
        }
        *(double2 *)(dst + j * kPlaneBlock) = double2{d[0], d[1]};
        *(double2 *)(dst + j * kPlaneBlock + 2) = double2{d[2], d[3]};
    }
}

// ---------------------------------------------------------------------------------------
// GEMM over the planes: 64 x 64 output tile, 4 waves of 32 x 32 (2 x 2 blocks of 16 x 16).
// ---------------------------------------------------------------------------------------
template <int NX>
struct PlaneTile {
    static constexpr int P_BYTES = kPlaneBlock * 8, X_BYTES = NX * kPlaneBlock * 8;
    static constexpr int STAGE = P_BYTES + X_BYTES;
    // 64 KB of stages per workgroup for one and three limbs (two workgroups per CU), 80 KB for four
    static constexpr int NBUF = NX == 1 ? 4 : 2;
    static constexpr int P_CHUNKS = P_BYTES / 16, X_CHUNKS = X_BYTES / 16;
};

template <int NX, bool FOLD, bool TRUNC>
__global__ __launch_bounds__(kThreads, 2) void gemm_f64_planes_kernel(const GemmArgs args) {
    using T = PlaneTile<NX>;
    static_assert(!TRUNC || (NX == 1 && !FOLD), "truncation: one limb, no fold");
    __shared__ __attribute__((aligned(16))) int8_t lds[T::NBUF * T::STAGE];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave_u >> 1, wn = wave_u & 1;
    const int total = args.tiles_m * args.tiles_n;
    int rb, cb;
    map_tile(blockIdx.x, total, args.n_xcd, args.tiles_m, args.tiles_n, args.group_m, rb, cb);
    const int si = find_seg(args, cb);
    const Seg &sg = args.seg[si];
    const uint64_t q = sg.q;
    const double qd = (double)q, qinv = sg.qinv;
    const int64_t m0 = (int64_t)rb * kPlaneBM;
    const int64_t n0 = (int64_t)(cb - sg.tile_begin) * kPlaneBN;
    const int KB = args.kblocks;
    const int8_t *gP = args.Pd + (int64_t)rb * KB * T::P_BYTES;
    const int8_t *gX = args.Xd + (int64_t)cb * KB * T::X_BYTES;

    v4d acc[2][2][NX];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int j = 0; j < NX; ++j) acc[a][b][j] = v4d{0.0, 0.0, 0.0, 0.0};
    uint64_t part[FOLD ? 2 : 1][FOLD ? 2 : 1][FOLD ? 4 : 1];
    if constexpr (FOLD) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) part[a][b][i] = 0;
    }

    // the buffer form of the direct-to-LDS load: the compiler counts it in vmcnt only, so the
    // MFMAs wait for just the fragment reads they use (the host keeps KB X_BYTES below 2^32)
    const __amdgpu_buffer_rsrc_t rsP = lds_src_rsrc(gP), rsX = lds_src_rsrc(gX);
    auto gload = [&](int kb, int buf) {
        int8_t *dst = lds + buf * T::STAGE;
        copy_to_lds_buf<kThreads, T::P_CHUNKS>(rsP, (uint32_t)kb * (uint32_t)T::P_BYTES, dst, tid, wave_u);
        copy_to_lds_buf<kThreads, T::X_CHUNKS>(rsX, (uint32_t)kb * (uint32_t)T::X_BYTES, dst + T::P_BYTES, tid,
                                               wave_u);
    };
    const int loads_per_stage = loads_of_wave<kThreads, T::P_CHUNKS>(wave_u) +
                                loads_of_wave<kThreads, T::X_CHUNKS>(wave_u);

    // One K step (4 of the 16 K of a stage): lane l holds A[row l%16][k l/16] of each
    // 16 x 4 plaintext block and B[k l/16][col l%16] of each 4 x 16 limb block.
    struct Frags {
        double a[2];
        double b[2][NX];
    };
    const int kr = lane >> 4, li = lane & 15;
    auto read_frags = [&](Frags &f, int buf, int kk) {
        const double *lp = (const double *)(lds + buf * T::STAGE);
        const double *lx = (const double *)(lds + buf * T::STAGE + T::P_BYTES);
        const int kl = kk * 4 + kr;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) f.a[mb] = lp[kl * kPlaneBM + wm * 32 + mb * 16 + li];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int j = 0; j < NX; ++j) f.b[nb][j] = lx[j * kPlaneBlock + kl * kPlaneBN + wn * 32 + nb * 16 + li];
    };
    auto mfmas = [&](const Frags &f) {
#pragma unroll
        for (int j = 0; j < NX; ++j)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    acc[mb][nb][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[mb], f.b[nb][j], acc[mb][nb][j], 0, 0, 0);
    };
    // sum_j c_j 2^{w j} mod q by Horner from the top limb, every c_j an exact integer
    auto recombine = [&](int a, int b, int i) -> uint64_t {
        uint64_t r = reduce_fp(acc[a][b][NX - 1][i], q, qd, qinv);
#pragma unroll
        for (int j = NX - 2; j >= 0; --j)
            r = addmod(mulmod_shoup(r, sg.wmod, sg.wshoup, q), reduce_fp(acc[a][b][j][i], q, qd, qinv), q);
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
                for (int j = 0; j < NX; ++j) acc[a][b][j] = v4d{0.0, 0.0, 0.0, 0.0};
    };

    // Pipeline (per wave): the fragments of the next K step are read while the MFMAs of the
    // current one run; at the last K step of a stage each wave waits for its own loads of the
    // next stage, the barrier makes all of them visible (and tells that every wave has read
    // the current buffer), the current buffer is refilled NBUF stages ahead, and the next
    // stage's first fragments are read before the last MFMAs of this one.
    auto outstanding = [&](int need, int issued_hi) {
        const int ahead = min(KB - 1, issued_hi) - need;
        return ahead > 0 ? ahead * loads_per_stage : 0;
    };
#pragma unroll
    for (int st = 0; st < T::NBUF; ++st)
        if (st < KB) gload(st, st);
    wait_vmcnt(outstanding(0, T::NBUF - 1));
    stage_barrier();
    Frags f0, f1;
    settle_scalar_loads();
    read_frags(f0, 0, 0);
#pragma unroll 1
    for (int kb = 0; kb < KB; ++kb) {
        const int cur = kb % T::NBUF;
        read_frags(f1, cur, 1);
        mfmas(f0);
        read_frags(f0, cur, 2);
        mfmas(f1);
        read_frags(f1, cur, 3);
        mfmas(f0);
        wait_lds_after_mfmas();
        wait_vmcnt(outstanding(kb + 1, kb + T::NBUF - 1));
        stage_barrier();
        if (kb + T::NBUF < KB) gload(kb + T::NBUF, cur);
        if (kb + 1 < KB) read_frags(f0, (kb + 1) % T::NBUF, 0);
        mfmas(f1);
        if constexpr (FOLD) {
            if ((kb + 1) % args.kfold == 0 && kb + 1 < KB) fold();
        }
    }

#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // 16x16 FP64 accumulator layout: column = lane % 16, row = 4 i + lane / 16
                const int64_t row = m0 + wm * 32 + a * 16 + 4 * i + kr;
                const int64_t col = n0 + wn * 32 + b * 16 + li;
                uint64_t v;
                if constexpr (TRUNC) v = reduce_fp(acc[a][b][0][i], q, qd, qinv);  // |acc| < q 2^51
                else v = recombine(a, b, i);
                if constexpr (FOLD) v = addmod(v, part[a][b][i], q);
                if (row < args.m && col < sg.n) sg.C[row * sg.ldc + col] = v;
            }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
int64_t f64_plane_bytes_p(int64_t tiles_m, int64_t kblocks) { return tiles_m * kblocks * kPlaneBlock * 8; }
int64_t f64_plane_bytes_x(int nx, int64_t tiles_n, int64_t kblocks) { return tiles_n * kblocks * nx * kPlaneBlock * 8; }

hipError_t launch_prep_p_planes(const int64_t *P, int64_t ldp, int64_t m, int64_t k, int tiles, int kblocks,
                                double *out, hipStream_t s) {
    if (tiles <= 0 || kblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_p_planes, dim3(tiles * kblocks), dim3(kThreads), 0, s, P, ldp, m, k, kblocks, out);
    return hipGetLastError();
}

hipError_t launch_prep_x_planes(int nx, bool trunc, const uint64_t *X, int64_t ldx, int64_t k, int64_t n, int tiles,
                                int kblocks, int w, uint64_t q, double *out, hipStream_t s) {
    if (tiles <= 0 || kblocks <= 0) return hipSuccess;
    const dim3 g(tiles * kblocks), b(kThreads);
    if (trunc && nx == 1) hipLaunchKernelGGL((prep_x_planes<1, true>), g, b, 0, s, X, ldx, k, n, kblocks, w, q, out);
    else if (!trunc && nx == 3) hipLaunchKernelGGL((prep_x_planes<3, false>), g, b, 0, s, X, ldx, k, n, kblocks, w, q, out);
    else if (!trunc && nx == 4) hipLaunchKernelGGL((prep_x_planes<4, false>), g, b, 0, s, X, ldx, k, n, kblocks, w, q, out);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int NX, bool FOLD, bool TRUNC>
static hipError_t launch_planes_t(const GemmArgs &a, hipStream_t s) {
    const int grid = a.tiles_m * a.tiles_n;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_f64_planes_kernel<NX, FOLD, TRUNC>), dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm_f64_planes(int nx, bool trunc, const GemmArgs &a, hipStream_t s) {
    const bool fold = a.kfold < a.kblocks;
    if (trunc) return (nx == 1 && !fold) ? launch_planes_t<1, false, true>(a, s) : hipErrorInvalidValue;
    if (nx == 3) return fold ? launch_planes_t<3, true, false>(a, s) : launch_planes_t<3, false, false>(a, s);
    if (nx == 4) return fold ? launch_planes_t<4, true, false>(a, s) : launch_planes_t<4, false, false>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace hlb
