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
// Contents: digit-split kernels (single problem and batched), the per-tile GEMM body, the
// grid kernel of one CP-MM / Mod-PP-MM, and the persistent kernel of a batch.
#include "common.hpp"
#include "launch.hpp"

namespace hlb {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

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
// Limb GEMM tile.
//   A workgroup of WAVES_M x WAVES_N waves computes a BM x BN output tile (BM = 32*WAVES_M,
//   BN = 32*WAVES_N); each wave owns one 32 x 32 block with NS int32 accumulators per output
//   (one per shift), i.e. 16*NS accumulator registers per lane.  K advances 64 bytes per LDS
//   stage (two MFMA K steps of 32).
// ---------------------------------------------------------------------------------------
template <int DP_, int DX_, int WAVES_M_, int WAVES_N_>
struct I8Tile {
    static constexpr int DP = DP_, DX = DX_, WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
    static constexpr int NS = DP + DX - 1;
    static constexpr int THREADS = 64 * WAVES_M * WAVES_N;
    static constexpr int BM = 32 * WAVES_M, BN = 32 * WAVES_N;
    static constexpr int P_TILE = DP * BM * kBK8;
    static constexpr int X_TILE = DX * BN * kBK8;
    static constexpr int STAGE = P_TILE + X_TILE;
    static constexpr int P_CHUNKS = P_TILE / 16, X_CHUNKS = X_TILE / 16;
    static_assert(P_CHUNKS % 64 == 0 && X_CHUNKS % 64 == 0, "tiles are whole wave loads");
    // Three LDS stages when they fit: global loads then have two stages of compute to land.
    static constexpr int NBUF = 3 * STAGE <= 160 * 1024 ? 3 : 2;
    static constexpr int LDS = NBUF * STAGE;
};

// Tile classes (8 waves each): class 0 = 128 x 64 outputs, class 1 = 64 x 128 outputs.
template <int DP, int DX> using Class0 = I8Tile<DP, DX, 4, 2>;
template <int DP, int DX> using Class1 = I8Tile<DP, DX, 2, 4>;

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

// Copies CHUNKS 16-byte chunks from global memory to LDS with the gfx950 direct-to-LDS
// load: lane l of a wave writes its 16 bytes at (wave-uniform LDS base) + 16 l, so the
// linear chunk order of the tile-major workspace arrives unchanged and no staging
// registers are used.  Chunks are dealt to waves in runs of 64.
template <int THREADS, int CHUNKS>
__device__ __forceinline__ void copy_to_lds(const int8_t *src, int8_t *dst, int tid, int wave_u) {
#pragma unroll
    for (int i = 0; i < (CHUNKS + THREADS - 1) / THREADS; ++i) {
        const int base = i * THREADS + wave_u * 64;  // wave-uniform
        if (CHUNKS % THREADS == 0 || base < CHUNKS)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)(src + (i * THREADS + tid) * 16),
                (__attribute__((address_space(3))) void *)(dst + base * 16), 16, 0, 0);
    }
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
        default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
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

    auto gload = [&](int kb, int buf) {
        int8_t *dp = lds + buf * T::STAGE;
        copy_to_lds<T::THREADS, T::P_CHUNKS>(job.gP + (int64_t)kb * T::P_TILE, dp, tid, wave_u);
        copy_to_lds<T::THREADS, T::X_CHUNKS>(job.gX + (int64_t)kb * T::X_TILE, dp + T::P_TILE, tid, wave_u);
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
        v4i b[T::DX];
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
        for (int j = 0; j < T::DX; ++j) f.b[j] = *(const v4i *)(lx + j * T::BN * 64 + xoff);
    };
    auto mfmas = [&](const Frags &f) {
#pragma unroll
        for (int i = 0; i < T::DP; ++i)
#pragma unroll
            for (int j = 0; j < T::DX; ++j)
                acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[i], f.b[j], acc[i + j], 0, 0, 0);
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
    read_frags(f0, 0, 0);
#pragma unroll 1
    for (int kb = 0; kb < KB; ++kb) {
        const int cur = kb % NBUF;
        read_frags(f1, cur, 1);
        mfmas(f0);
        interleave_reads_with_mfmas<T::DP + T::DX>();
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
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
