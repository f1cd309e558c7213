// i8_tile.hpp -- the INT8 limb-GEMM tile shared by the exact and truncated launchers.
//
// Strategy 1 of Section 6.1 (Lemma le:strategy1, Eq decomp) with base K = 256 and balanced
// signed digits: every digit-plane pair P_i * X_j is multiplied exactly on
// v_mfma_i32_32x32x32_i8 and accumulated into the int32 accumulator of its shift s = i + j;
// the epilogue recombines sum_s c_s 256^s and reduces it modulo q.  A tile may drop the
// products of the lowest shifts (the truncation of Strategy 2, keeping only the high-order
// terms of the decomposition); with DROP = 0 it is exact.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace hlb {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------------------
// Limb GEMM tile.
//   A workgroup of WAVES_M x WAVES_N waves computes a BM x BN output tile (BM = 32*WAVES_M,
//   BN = 32*WAVES_N); each wave owns one 32 x 32 block with NS int32 accumulators per output
//   (one per shift), i.e. 16*NS accumulator registers per lane.  K advances 64 bytes per LDS
//   stage (two MFMA K steps of 32).
// ---------------------------------------------------------------------------------------
template <int DP_, int DX_, int WAVES_M_, int WAVES_N_, int DROP_ = 0>
struct I8Tile {
    static constexpr int DP = DP_, DX = DX_, WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
    static constexpr int NS = DP + DX - 1;
    // Products P_i X_j with i + j < DROP are skipped; X digits below J0 then take part in no
    // product and are not loaded.
    static constexpr int DROP = DROP_;
    static constexpr int J0 = DROP > DP - 1 ? DROP - (DP - 1) : 0;
    static_assert(DROP >= 0 && J0 < DX, "at least one product per X digit range");
    static constexpr int THREADS = 64 * WAVES_M * WAVES_N;
    static constexpr int BM = 32 * WAVES_M, BN = 32 * WAVES_N;
    static constexpr int P_TILE = DP * BM * kBK8;
    static constexpr int X_TILE = DX * BN * kBK8;         // workspace bytes per stage
    static constexpr int X_LDS = (DX - J0) * BN * kBK8;   // bytes of it loaded into LDS
    static constexpr int STAGE = P_TILE + X_LDS;
    static constexpr int P_CHUNKS = P_TILE / 16, X_CHUNKS = X_LDS / 16;
    static_assert(P_CHUNKS % 64 == 0 && X_CHUNKS % 64 == 0, "tiles are whole wave loads");
    // Three LDS stages when they fit: global loads then have two stages of compute to land.
    static constexpr int NBUF = 3 * STAGE <= 160 * 1024 ? 3 : 2;
    static constexpr int LDS = NBUF * STAGE;
};

// Tile classes (8 waves each): class 0 = 128 x 64 outputs, class 1 = 64 x 128 outputs.
template <int DP, int DX, int DROP = 0> using Class0 = I8Tile<DP, DX, 4, 2, DROP>;
template <int DP, int DX, int DROP = 0> using Class1 = I8Tile<DP, DX, 2, 4, DROP>;

// Exact integer value sum_s acc[s] 256^s reduced mod q, by Horner from the top shift:
// r <- (256 r + c_s) mod q with r < q < 2^52 and |c_s| < 2^31, so every intermediate fits
// in int64 and |t/q| < 2^31 meets the precondition of reduce_near.
template <int NS>
__device__ __forceinline__ uint64_t recombine_i8(const int (&c)[NS], uint64_t q, double qinv) {
    uint64_t r = reduce_near((int64_t)c[NS - 1], q, qinv);
#pragma unroll
    for (int s = NS - 2; s >= 0; --s) r = reduce_near((int64_t)(r << 8) + (int64_t)c[s], q, qinv);
    return r;
}

// Everything one output tile needs.
struct TileJob {
    const int8_t *gP;  // first K block of this tile row's plaintext digits
    const int8_t *gX;  // first K block of this tile column's ciphertext digits
    int KB;            // K blocks
    int kfold;         // K blocks accumulated before a fold
    int64_t row0, m;   // first output row of the tile, valid rows of the problem
    int64_t col0, n;   // first output column (within its segment), valid columns
    uint64_t *C;
    int64_t ldc;
    uint64_t q;
    double qinv;
};

// One output tile: K loop with the LDS pipeline, then the fused recombination / mod-q
// epilogue.  On return no LDS access of this tile is outstanding.
template <class T, bool FOLD>
__device__ __forceinline__ void run_tile(const TileJob &job, int8_t *lds) {
    constexpr int NBUF = T::NBUF;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave_u / T::WAVES_N, wn = wave_u % T::WAVES_N;
    const uint64_t q = job.q;
    const double qinv = job.qinv;

    v16i acc[T::NS];
#pragma unroll
    for (int s = 0; s < T::NS; ++s) acc[s] = v16i{0};
    // running residues of folded K chunks (only materialised when FOLD)
    uint64_t part[FOLD ? 16 : 1];
    if constexpr (FOLD) {
#pragma unroll
        for (int r = 0; r < 16; ++r) part[r] = 0;
    }

    // the buffer form of the direct-to-LDS load: the compiler counts it in vmcnt only, so the
    // MFMAs wait for just the fragment reads they use (byte offsets within a tile's panels stay
    // below 2^32: KB P_TILE and KB X_TILE are at most a few hundred MiB)
    const __amdgpu_buffer_rsrc_t rsP = lds_src_rsrc(job.gP), rsX = lds_src_rsrc(job.gX + T::J0 * T::BN * kBK8);
    auto gload = [&](int kb, int buf) {
        int8_t *dp = lds + buf * T::STAGE;
        copy_to_lds_buf<T::THREADS, T::P_CHUNKS>(rsP, (uint32_t)kb * (uint32_t)T::P_TILE, dp, tid, wave_u);
        copy_to_lds_buf<T::THREADS, T::X_CHUNKS>(rsX, (uint32_t)kb * (uint32_t)T::X_TILE, dp + T::P_TILE, tid, wave_u);
    };
    const int loads_per_stage = loads_of_wave<T::THREADS, T::P_CHUNKS>(wave_u) +
                                loads_of_wave<T::THREADS, T::X_CHUNKS>(wave_u);

    // fragment addresses: this lane's row of the P tile and column of the X tile
    const int prow = wm * 32 + (lane & 31);
    const int xcol = wn * 32 + (lane & 31);
    // One K half (32 bytes) of a stage: the DP plaintext and DX ciphertext fragments of this
    // lane, then the DP x DX digit-pair MFMAs into the shift accumulators.
    struct Frags {
        v4i a[T::DP];
        v4i b[T::DX - T::J0];  // X digits J0 .. DX-1
    };
    auto read_frags = [&](Frags &f, int buf, int kk) {
        const int8_t *lp = lds + buf * T::STAGE;
        const int8_t *lx = lp + T::P_TILE;
        const int c = kk * 2 + (lane >> 5);
        const int poff = prow * 64 + ((c ^ swz(prow)) << 4);
        const int xoff = xcol * 64 + ((c ^ swz(xcol)) << 4);
#pragma unroll
        for (int i = 0; i < T::DP; ++i) f.a[i] = *(const v4i *)(lp + i * T::BM * 64 + poff);
#pragma unroll
        for (int j = 0; j < T::DX - T::J0; ++j) f.b[j] = *(const v4i *)(lx + j * T::BN * 64 + xoff);
    };
    auto mfmas = [&](const Frags &f) {
#pragma unroll
        for (int i = 0; i < T::DP; ++i)
#pragma unroll
            for (int j = T::J0; j < T::DX; ++j)
                if (i + j >= T::DROP)
                    acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[i], f.b[j - T::J0], acc[i + j], 0, 0, 0);
    };
    auto fold = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int c[T::NS];
#pragma unroll
            for (int s = 0; s < T::NS; ++s) c[s] = acc[s][r];
            part[r] = addmod(part[r], recombine_i8<T::NS>(c, q, qinv), q);
        }
#pragma unroll
        for (int s = 0; s < T::NS; ++s) acc[s] = v16i{0};
    };

    // Pipeline (per wave), half a stage deep in registers and NBUF stages deep in LDS:
    //   read F1 = (kb, second half) | MFMAs on F0 | wait: F1 read, stage kb+1 landed |
    //   barrier | DMA stage kb+NBUF into the buffer of stage kb | read F0 = (kb+1, first half) |
    //   MFMAs on F1
    // so every LDS read overlaps a half stage of MFMAs, and every stage's global loads have
    // NBUF-1 stages of compute to land.  At the barrier all waves have finished reading the
    // buffer of stage kb (hence it can be refilled) and have seen stage kb+1 land.
    const int KB = job.KB;
    // loads still allowed in flight when stage `need` must have landed, given that stages
    // up to min(KB-1, issued_hi) have been issued
    auto outstanding = [&](int need, int issued_hi) {
        const int ahead = min(KB - 1, issued_hi) - need;
        return ahead > 0 ? ahead * loads_per_stage : 0;
    };
#pragma unroll
    for (int st = 0; st < NBUF; ++st)
        if (st < KB) gload(st, st);
    wait_vmcnt(outstanding(0, NBUF - 1));
    stage_barrier();
    Frags f0, f1;
    settle_scalar_loads();
    read_frags(f0, 0, 0);
#pragma unroll 1
    for (int kb = 0; kb < KB; ++kb) {
        const int cur = kb % NBUF;
        read_frags(f1, cur, 1);
        mfmas(f0);
        interleave_reads_with_mfmas<T::DP + T::DX - T::J0>();
        wait_lds_after_mfmas();
        // stages issued so far: up to kb + NBUF - 1
        wait_vmcnt(outstanding(kb + 1, kb + NBUF - 1));
        stage_barrier();
        if (kb + NBUF < KB) gload(kb + NBUF, cur);
        if (kb + 1 < KB) read_frags(f0, (kb + 1) % NBUF, 0);
        mfmas(f1);
        if constexpr (FOLD) {
            if ((kb + 1) % job.kfold == 0 && kb + 1 < KB) fold();
        }
    }

    // Epilogue: recombine, reduce, write canonical residues (row- and column-masked).
    const int64_t row0 = job.row0 + wm * 32;
    const int64_t col = job.col0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        // 32x32 accumulator layout: column = lane % 32, row = 8 (r / 4) + 4 (lane / 32) + r % 4
        const int64_t row = row0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        int c[T::NS];
#pragma unroll
        for (int s = 0; s < T::NS; ++s) c[s] = acc[s][r];
        uint64_t v = recombine_i8<T::NS>(c, q, qinv);
        if constexpr (FOLD) v = addmod(v, part[r], q);
        if (row < job.m && col < job.n) job.C[row * job.ldc + col] = v;
    }
}

// ---------------------------------------------------------------------------------------
// Grid kernel of one problem: one workgroup per output tile (XCD-aware raster).
// ---------------------------------------------------------------------------------------
template <class T, bool FOLD>
__global__ __launch_bounds__(T::THREADS, 1) void gemm_i8_kernel(const GemmArgs args) {
    __shared__ __attribute__((aligned(16))) int8_t lds[T::LDS];
    const int total = args.tiles_m * args.tiles_n;
    int rb, cb;
    map_tile(blockIdx.x, total, args.n_xcd, args.tiles_m, args.tiles_n, args.group_m, rb, cb);
    const int si = find_seg(args, cb);
    const Seg &sg = args.seg[si];
    TileJob job;
    job.gP = args.Pd + (int64_t)rb * args.kblocks * T::P_TILE;
    job.gX = args.Xd + (int64_t)cb * args.kblocks * T::X_TILE;
    job.KB = args.kblocks;
    job.kfold = args.kfold;
    job.row0 = (int64_t)rb * T::BM;
    job.m = args.m;
    job.col0 = (int64_t)(cb - sg.tile_begin) * T::BN;
    job.n = sg.n;
    job.C = sg.C;
    job.ldc = sg.ldc;
    job.q = sg.q;
    job.qinv = sg.qinv;
    run_tile<T, FOLD>(job, lds);
}

template <class T, bool FOLD>
static hipError_t launch_gemm_t(const GemmArgs &a, hipStream_t s) {
    const int grid = a.tiles_m * a.tiles_n;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_i8_kernel<T, FOLD>), dim3(grid), dim3(T::THREADS), 0, s, a);
    return hipGetLastError();
}

template <class T>
static hipError_t launch_gemm_fold(const GemmArgs &a, hipStream_t s) {
    return a.kfold < a.kblocks ? launch_gemm_t<T, true>(a, s) : launch_gemm_t<T, false>(a, s);
}


}  // namespace hlb
