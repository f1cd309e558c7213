// crt.hip -- multimodular (CRT) INT8 form of the exact Mod-PP-MM / CP-MM on gfx950.
//
// Strategy 3 of Section 6.1 in its FLINT variant (lift the operands to integers, compute the
// product modulo small coprime moduli, recombine by the CRT), with the moduli chosen so that
// every modular product is one exact INT8 -> INT32 matrix product:
//   1. split: the centred operands (plaintext as signed integers; residues x mod q taken in
//      (-q/2, q/2]) become D planes of balanced residues modulo p_0 .. p_{D-1} <= 256, in the
//      tile-major, swizzled layout of the digit split ([tile][k block][plane][128][64]);
//   2. GEMM: one plain INT8 product per modulus and output tile (v_mfma_i32_32x32x32_i8,
//      64 x 64 outputs per wave), |c| <= k 2^14 < 2^31; the epilogue writes the byte
//      y_i = c * (M / p_i)^{-1} mod p_i;
//   3. combine: V = sum_i y_i (M / p_i) - t M with t = round(sum_i y_i / p_i) is the exact
//      integer product as long as M > 2 |V|, and V mod q is formed from w_i = (M / p_i) mod q.
// D moduli replace the DP * DX digit products of Strategy 1 (11 instead of 21 for a 20-bit
// plaintext and 50-bit primes at k = 8192; 15 instead of 49 for two full residue operands).
#include "common.hpp"
#include "crt.hpp"
#include "launch.hpp"

namespace hlb {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------------------
// 1. Residue split, straight from registers to the workspace (no LDS): one thread owns one
//    16-byte chunk (16 consecutive K) of one row of a 128-row tile -- a row of P, or a
//    column of X -- and writes that chunk of every plane at its swizzled position.  Lanes
//    run over the 4 chunks of a row first, so each 4 lanes store one contiguous 64-byte row.
//    Values are taken as signed integers (qc = 0) or as residues modulo qc in their centred
//    representatives; entries outside the valid range become zero.
// ---------------------------------------------------------------------------------------
constexpr int kCrtR = 128;  // rows (columns) per split tile

template <int D>
__device__ __forceinline__ void crt_store_chunk(const double (&v)[16], int8_t *blk, int r, int c) {
    // blk: the [D][128][64] block of this (tile, k block); row r, logical chunk c
    int8_t *dst = blk + r * 64 + ((c ^ swz(r)) << 4);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        uint32_t w[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            uint32_t x = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                x |= ((uint32_t)balanced_residue(v[q4 * 4 + e], kCrtModuli[i]) & 0xffu) << (8 * e);
            w[q4] = x;
        }
        *(uint4 *)(dst + i * kCrtR * 64) = uint4{w[0], w[1], w[2], w[3]};
    }
}

__device__ __forceinline__ double crt_centred(uint64_t x, uint64_t qc) {
    const int64_t s = (qc != 0 && 2 * x > qc) ? (int64_t)x - (int64_t)qc : (int64_t)x;
    return (double)s;
}

// grid: (tiles * kblocks) workgroups of 512 threads = 128 rows x 4 chunks
template <int D>
__global__ __launch_bounds__(512) void crt_split_rows(const int64_t *__restrict__ P, int64_t ldp, int64_t m,
                                                      int64_t k, int kblocks, uint64_t qc, int8_t *__restrict__ out) {
    const int tile = blockIdx.x / kblocks, kb = blockIdx.x % kblocks;
    const int r = threadIdx.x >> 2, c = threadIdx.x & 3;
    const int64_t row = (int64_t)tile * kCrtR + r;
    const int64_t k0 = (int64_t)kb * kBK8 + c * 16;
    const int64_t rc = row < m ? row : m - 1;
    uint64_t x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = (uint64_t)P[rc * ldp + (k0 + e < k ? k0 + e : k - 1)];
#pragma unroll
    for (int e = 0; e < 16; ++e) asm volatile("" : "+v"(x[e]));  // all loads issued before the masks
    double v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = (row < m && k0 + e < k) ? crt_centred(x[e], qc) : 0.0;
    crt_store_chunk<D>(v, out + ((int64_t)tile * kblocks + kb) * (D * kCrtR * kBK8), r, c);
}

template <int D>
__global__ __launch_bounds__(512) void crt_split_cols(const uint64_t *__restrict__ X, int64_t ldx, int64_t k,
                                                      int64_t n, int kblocks, uint64_t qc, int8_t *__restrict__ out) {
    const int tile = blockIdx.x / kblocks, kb = blockIdx.x % kblocks;
    const int r = threadIdx.x >> 2, c = threadIdx.x & 3;
    const int64_t col = (int64_t)tile * kCrtR + r;
    const int64_t k0 = (int64_t)kb * kBK8 + c * 16;
    const int64_t cc = col < n ? col : n - 1;
    uint64_t x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = X[(k0 + e < k ? k0 + e : k - 1) * ldx + cc];
#pragma unroll
    for (int e = 0; e < 16; ++e) asm volatile("" : "+v"(x[e]));
    double v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = (col < n && k0 + e < k) ? crt_centred(x[e], qc) : 0.0;
    crt_store_chunk<D>(v, out + ((int64_t)tile * kblocks + kb) * (D * kCrtR * kBK8), r, c);
}

// ---------------------------------------------------------------------------------------
// 2. One INT8 product per modulus on a 256 x BN output tile: WM x WN waves, each owning
//    MB x NB blocks of 32 x 32 outputs (WM * MB * 32 = 256).  Variants (tile, waves, block
//    per wave): 256 x 128 with 8 waves of 64 x 64; 256 x 256 with 8 waves of 64 x 128.
//    (A wave of 128 x 128 would need 256 accumulator registers plus its fragments, more than
//    the register file holds without spilling in the main loop.)
// ---------------------------------------------------------------------------------------
constexpr int kCrtBM = 256;
constexpr int kCrtSub = kCrtR * kBK8;  // bytes of one plane block (128 x 64)

// A stage holds only MB * NB MFMAs per wave and K half, so several stages must be in flight
// to cover the load latency: as many as fit in the 160 KB of LDS.
template <int MB_, int NB_, int WM_, int WN_>
struct CrtTile {
    static constexpr int MB = MB_, NB = NB_, WM = WM_, WN = WN_;
    static_assert(WM * MB * 32 == kCrtBM, "256 rows per tile");
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int BN = WN * NB * 32;
    static constexpr int XSUB = BN / kCrtR;            // residue plane blocks per stage
    static constexpr int STAGE = (2 + XSUB) * kCrtSub;  // two plaintext blocks + residue blocks
    static constexpr int GROUP = 2;                      // stages per barrier
    static constexpr int NBUF = (160 * 1024) / STAGE / GROUP * GROUP;
};
using CrtNarrow = CrtTile<2, 2, 4, 2>;
using CrtWide = CrtTile<2, 4, 4, 2>;

__device__ __forceinline__ uint8_t crt_y(int c, int p, int inv) {
    // (c mod p) * inv mod p, in [0, p); c and the products are exact in double
    const double pd = (double)p, pinv = 1.0 / pd;
    double r = __builtin_fma(-__builtin_floor((double)c * pinv), pd, (double)c);
    r = r < 0.0 ? r + pd : r;
    r = r >= pd ? r - pd : r;
    double y = r * (double)inv;
    y = __builtin_fma(-__builtin_floor(y * pinv), pd, y);
    y = y < 0.0 ? y + pd : y;
    y = y >= pd ? y - pd : y;
    return (uint8_t)(int)y;
}

template <class T>
__global__ __launch_bounds__(T::THREADS, 1) void crt_gemm_kernel(const CrtGemmArgs args) {
    constexpr int MB = T::MB, NB = T::NB, kCrtThreads = T::THREADS, kCrtWavesN = T::WN;
    constexpr int kCrtNbuf = T::NBUF;
    __shared__ __attribute__((aligned(16))) int8_t lds[kCrtNbuf * T::STAGE];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave_u / kCrtWavesN, wn = wave_u % kCrtWavesN;

    // the D moduli stack as D row bands of one (D * tiles_m) x tiles_n grid
    const int total = args.D * args.tiles_m * args.tiles_n;
    int rbv, cb;
    map_tile(blockIdx.x, total, args.n_xcd, args.D * args.tiles_m, args.tiles_n, args.group_m, rbv, cb);
    const int mi = rbv / args.tiles_m, rb = rbv % args.tiles_m;
    int si = 0;
#pragma unroll 1
    for (int i = 1; i < args.nseg; ++i)
        if (cb >= args.seg[i].tile_begin) si = i;
    const CrtSeg &sg = args.seg[si];

    const int KB = args.kblocks;
    const int64_t plane_stride = (int64_t)args.D * kCrtSub;  // bytes of one k block of a 128-wide tile
    const int64_t tile_stride = (int64_t)KB * plane_stride;  // bytes of one 128-wide tile
    const int8_t *gP = args.Pd + (int64_t)(2 * rb) * tile_stride + (int64_t)mi * kCrtSub;
    const int8_t *gX = args.Xd + (int64_t)(cb * T::XSUB) * tile_stride + (int64_t)mi * kCrtSub;

    v16i acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = v16i{0};

    constexpr int CH = kCrtSub / 16;  // 16-byte chunks per block
    auto gload = [&](int kb, int buf) {
        int8_t *dst = lds + buf * T::STAGE;
        const int64_t off = (int64_t)kb * plane_stride;
#pragma unroll
        for (int b = 0; b < 2; ++b) copy_to_lds<kCrtThreads, CH>(gP + b * tile_stride + off, dst + b * kCrtSub, tid, wave_u);
#pragma unroll
        for (int b = 0; b < T::XSUB; ++b)
            copy_to_lds<kCrtThreads, CH>(gX + b * tile_stride + off, dst + (2 + b) * kCrtSub, tid, wave_u);
    };
    const int loads_per_stage = (2 + T::XSUB) * loads_of_wave<kCrtThreads, CH>(wave_u);

    // plaintext rows of this wave: wm * 32 MB + 32 mb + lane % 32, in 128-row block psub;
    // residue columns: wn * 32 NB + 32 nb + lane % 32, in block (that) / 128
    const int psub = (wm * 32 * MB) / kCrtR;
    const int prow0 = (wm * 32 * MB) % kCrtR;
    struct Frags {
        v4i a[MB], b[NB];
    };
    auto read_frags = [&](Frags &f, int buf, int kk) {
        const int8_t *lp = lds + buf * T::STAGE + psub * kCrtSub;
        const int8_t *lx = lds + buf * T::STAGE + 2 * kCrtSub;
        const int c = kk * 2 + (lane >> 5);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int r = prow0 + mb * 32 + (lane & 31);
            f.a[mb] = *(const v4i *)(lp + r * 64 + ((c ^ swz(r)) << 4));
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int col = wn * 32 * NB + nb * 32 + (lane & 31);
            const int r = col & (kCrtR - 1);
            f.b[nb] = *(const v4i *)(lx + (col / kCrtR) * kCrtSub + r * 64 + ((c ^ swz(r)) << 4));
        }
    };
    auto mfmas = [&](const Frags &f) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[mb], f.b[nb], acc[mb][nb], 0, 0, 0);
    };

    // Pipeline: half a stage of fragments in registers, NBUF stages in LDS, and one wait +
    // barrier per group of G stages.  At a group's last half-stage each wave waits for its
    // own loads of the whole next group, the barrier makes them visible (and tells that every
    // wave has finished reading this group's buffers), and those buffers are refilled NBUF
    // stages ahead.
    constexpr int G = T::GROUP;
    auto outstanding = [&](int need_hi, int issued_hi) {
        const int ahead = min(KB - 1, issued_hi) - min(KB - 1, need_hi);
        return ahead > 0 ? ahead * loads_per_stage : 0;
    };
#pragma unroll
    for (int st = 0; st < kCrtNbuf; ++st)
        if (st < KB) gload(st, st);
    wait_vmcnt(outstanding(G - 1, kCrtNbuf - 1));
    stage_barrier();
    Frags f0, f1;
    read_frags(f0, 0, 0);
#pragma unroll 1
    for (int kb = 0; kb < KB; kb += G) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int st = kb + g;
            if (st >= KB) break;
            const int cur = st % kCrtNbuf;
            read_frags(f1, cur, 1);
            mfmas(f0);
            interleave_reads_with_mfmas<MB + NB>();
            if (g == G - 1 || st + 1 == KB) {
                wait_lds_after_mfmas();
                // stages issued so far: up to kb + NBUF - 1; the next group must have landed
                wait_vmcnt(outstanding(kb + 2 * G - 1, kb + kCrtNbuf - 1));
                stage_barrier();
#pragma unroll
                for (int h = 0; h < G; ++h)
                    if (kb + h + kCrtNbuf < KB) gload(kb + h + kCrtNbuf, (kb + h) % kCrtNbuf);
            }
            if (st + 1 < KB) read_frags(f0, (st + 1) % kCrtNbuf, 0);
            mfmas(f1);
        }
    }

    const int p = kCrtModuli[mi];
    const int inv = args.inv[mi];
    const int64_t m0 = (int64_t)rb * kCrtBM + wm * 32 * MB;
    const int64_t n0 = (int64_t)(cb - sg.tile_begin) * T::BN + wn * 32 * NB;
    uint8_t *Y = sg.Y + (int64_t)mi * args.m * sg.ldy;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                // 32x32 accumulator layout: column = lane % 32, row = 8 (r / 4) + 4 (lane / 32) + r % 4
                const int64_t row = m0 + mb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int64_t col = n0 + nb * 32 + (lane & 31);
                if (row < args.m && col < sg.n) Y[row * sg.ldy + col] = crt_y(acc[mb][nb][r], p, inv);
            }
}

// ---------------------------------------------------------------------------------------
// 3. Recombination
// ---------------------------------------------------------------------------------------
// x mod q for any x < 2^64 and q < 2^52 (Barrett with mu = floor(2^64 / q): the quotient
// estimate is at most two below floor(x / q), so two corrections finish).
__device__ __forceinline__ uint64_t reduce_u64(uint64_t x, uint64_t q, uint64_t mu) {
    uint64_t r = x - __umul64hi(x, mu) * q;
    r = r >= q ? r - q : r;
    return r >= q ? r - q : r;
}

// Thread: 4 consecutive columns of one row.  The D planes are read as one dword each (the
// plane rows are padded to 16 bytes), sum_i y_i w_i < 16 * 2^8 * 2^52 accumulates without
// reduction, and the rounding t = round(sum_i y_i / p_i) needs only single precision: the
// fraction lies within 1/4 of an integer, far beyond its rounding error.
__global__ __launch_bounds__(kThreads) void crt_combine_kernel(const CrtCombineArgs a) {
    const int64_t plane = a.m * a.ldy;
    for (int64_t row = blockIdx.y; row < a.m; row += gridDim.y) {
        for (int64_t c4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; c4 < a.n;
             c4 += (int64_t)gridDim.x * blockDim.x * 4) {
            const uint8_t *y = a.Y + row * a.ldy + c4;
            uint64_t s[4] = {0, 0, 0, 0};
            float f[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int i = 0; i < a.D; ++i) {
                const uint32_t v = *(const uint32_t *)(y + (int64_t)i * plane);
                const uint64_t w = a.w[i];
                const float pi = a.pinv[i];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t b = (v >> (8 * e)) & 0xffu;
                    s[e] += (uint64_t)b * w;
                    f[e] = __builtin_fmaf((float)b, pi, f[e]);
                }
            }
            uint64_t *out = a.C + row * a.ldc + c4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (c4 + e >= a.n) break;
                const uint64_t t = (uint64_t)__builtin_floorf(f[e] + 0.5f);
                const uint64_t sr = reduce_u64(s[e], a.q, a.barrett);
                const uint64_t tm = reduce_u64(t * a.Mq, a.q, a.barrett);
                out[e] = sr >= tm ? sr - tm : sr + a.q - tm;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
bool crt_supported_d(int D) { return D == 8 || D == 10 || D == 11 || D == 12 || D == 14 || D == 16; }

int crt_round_d(int D) {
    for (int d : {8, 10, 11, 12, 14, 16})
        if (D <= d) return d;
    return 0;
}

#define HLB_CRT_D(X) X(8) X(10) X(11) X(12) X(14) X(16)

hipError_t launch_crt_split_rows(int D, const int64_t *P, int64_t ldp, int64_t m, int64_t k, int tiles, int kblocks,
                                 uint64_t qc, int8_t *out, hipStream_t s) {
    if (tiles <= 0 || kblocks <= 0) return hipSuccess;
    const dim3 g(tiles * kblocks), b(512);
#define HLB_CASE(DD) \
    if (D == DD) { hipLaunchKernelGGL(crt_split_rows<DD>, g, b, 0, s, P, ldp, m, k, kblocks, qc, out); return hipGetLastError(); }
    HLB_CRT_D(HLB_CASE)
#undef HLB_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_crt_split_cols(int D, const uint64_t *X, int64_t ldx, int64_t k, int64_t n, int tiles, int kblocks,
                                 uint64_t qc, int8_t *out, hipStream_t s) {
    if (tiles <= 0 || kblocks <= 0) return hipSuccess;
    const dim3 g(tiles * kblocks), b(512);
#define HLB_CASE(DD) \
    if (D == DD) { hipLaunchKernelGGL(crt_split_cols<DD>, g, b, 0, s, X, ldx, k, n, kblocks, qc, out); return hipGetLastError(); }
    HLB_CRT_D(HLB_CASE)
#undef HLB_CASE
    return hipErrorInvalidValue;
}

int crt_tile_cols(int variant) { return variant == 0 ? CrtNarrow::BN : CrtWide::BN; }

template <class T>
static hipError_t launch_crt_t(int64_t grid, const CrtGemmArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(crt_gemm_kernel<T>, dim3((unsigned)grid), dim3(T::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_crt_gemm(int variant, const CrtGemmArgs &a, hipStream_t s) {
    const int64_t grid = (int64_t)a.D * a.tiles_m * a.tiles_n;
    if (grid <= 0) return hipSuccess;
    if (grid > INT32_MAX) return hipErrorInvalidValue;
    return variant == 0 ? launch_crt_t<CrtNarrow>(grid, a, s) : launch_crt_t<CrtWide>(grid, a, s);
}

hipError_t launch_crt_combine(const CrtCombineArgs &a, hipStream_t s) {
    if (a.m <= 0 || a.n <= 0) return hipSuccess;
    int64_t gx = (a.n + kThreads * 4 - 1) / (kThreads * 4);
    gx = gx > 1024 ? 1024 : gx;
    const int64_t gy = a.m > 65535 ? 65535 : a.m;
    hipLaunchKernelGGL(crt_combine_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace hlb
