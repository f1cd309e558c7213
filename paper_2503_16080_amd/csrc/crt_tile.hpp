// crt_tile.hpp -- the output tile of the multimodular (CRT) INT8 products on gfx950: one
// exact INT8 -> INT32 matrix product per small modulus (v_mfma_i32_32x32x32_i8) over a tile
// of the residue planes written by the splits, with the epilogue that reduces each product
// modulo its modulus and stores y_i = c mod p_i in the accumulator order of the product
// planes (crt.hpp).  Strategy 3 of Section 6.1 in its FLINT variant.  crt_tile runs one tile
// (one workgroup per tile, and the items of the batch GEMM, crt_gemm_batch.hip); crt_tiles runs
// the stream of tiles of a persistent workgroup (the GEMM of one call, crt_gemm.hip).
#pragma once

#include "common.hpp"
#include "crt.hpp"

namespace hlb {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------------------
// One INT8 product per modulus on a 256 x BN output tile: WM x WN waves, each owning
//    MB x NB blocks of 32 x 32 outputs (WM * MB * 32 = 256).  Variants (tile, waves, block
//    per wave): 256 x 128 with 8 waves of 64 x 64; 256 x 256 with 8 waves of 64 x 128;
//    256 x 384 with 8 waves of 128 x 96 (the default: 24 MFMAs per wave and stage, the most
//    that two waves per SIMD can hold accumulators for, with 12% fewer LDS bytes per MFMA than
//    64 x 128).  (Four waves of 128 x 128 need their 256 accumulators in AGPRs and leave one
//    wave per SIMD, which hides less latency: measured slower.)
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
using CrtWider = CrtTile<4, 3, 2, 4>;

// c mod p in [0, p) for any int32 c and p <= 256, in twelve full-rate operations:
//  * c = h 2^16 + l (h signed, 0 <= l < 2^16): u = h (2^16 mod p) + l = c (mod p) with
//    |u| < 2^23 + 2^16, one 24-bit multiply-add (|h| < 2^15, 2^16 mod p < 2^8);
//  * u is exact in single precision, and t = floor(u (1/p)) is within one of floor(u / p):
//    the product carries a relative error below 2^-23, so an absolute one below 2^-6;
//  * r = u - t p is formed exactly by one fused multiply-add (the exact value, in [-p, 2p),
//    is representable) and brought into [0, p) by two unsigned minima:
//    min(r, r + p) maps [-p, 0) to [0, p), and min(r, r - p) maps [p, 2p) to [0, p) (the other
//    operand wraps to a large unsigned value).
__device__ __forceinline__ uint32_t crt_y(int c, int p, int c16, float pinv) {
    // the 24-bit multiply-add written out: left to itself the compiler picks the quarter-rate
    // 64-bit multiply-add here
    int u;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(u) : "v"(c >> 16), "v"(c16), "v"(c & 0xffff));
    const float uf = (float)u;
    const float tf = __builtin_floorf(uf * pinv);
    const int r = (int)__builtin_fmaf(-tf, (float)p, uf);
    const uint32_t r1 = min((uint32_t)r, (uint32_t)(r + p));
    return min(r1, r1 - (uint32_t)p);
}

// c mod p in [0, p) in six full-rate operations when |c| <= 2^28 (a product over at most
// 2^14 of K, i.e. at most kCrtShortKB K blocks, of residues in [-128, 127]) and p >= 191 (every
// modulus of the table):
//  * x = c (1/p), with the conversion, the reciprocal and the product each rounded to
//    nearest in single precision, is within 3 2^-24 |c / p| <= 48 / p < 0.26 of c / p;
//  * so x + 1/2 (exact, or rounded to single precision: a change below 2^-3 at these
//    magnitudes) lies within (c / p, c / p + 1), and t = floor(x + 1/2) (one rounding
//    conversion) is floor(c / p) or one more; r = c - t p lies in [-p, p), and |t| < 2^21, so
//    one 24-bit multiply-add forms r exactly;
//  * one unsigned minimum maps [-p, 0) to [0, p), as in crt_y.
constexpr int kCrtShortKB = 256;
__device__ __forceinline__ uint32_t crt_y_short(int c, int negp, float pinv) {
    int t, r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(t) : "v"((float)c * pinv));
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(t), "v"(negp), "v"(c));
    return min((uint32_t)r, (uint32_t)(r - negp));
}

// Where the 32-column block column bc of a tile goes: the product-plane block of its first
// block row (1 KiB per 32 x 32 block) and the bytes from one block row to the next; null p
// for a column outside every output.
struct CrtBlockCol {
    uint8_t *p;
    int64_t row_bytes;
};

// The epilogue of a wave: its MB x NB blocks of 32 x 32 products reduced modulo p (by
// crt_y_short when SHORT, for tiles of at most kCrtShortKB K blocks; else by crt_y) and
// stored, one 16-byte store per block and lane, block column bc at dst(bc) (a wave-uniform
// CrtBlockCol).  Returns the stores issued.
template <int MB, int NB, bool SHORT, class Dst>
__device__ __forceinline__ int crt_epilogue(const v16i (&acc)[MB][NB], int p, int wm, int wn, int lane,
                                            const Dst &dst) {
    const int c16 = (1 << 16) % p;
    const float pinv = 1.0f / (float)p;
    int stores = 0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const CrtBlockCol col = dst(wn * NB + nb);
        if (!col.p) continue;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t y = SHORT ? crt_y_short(acc[mb][nb][e], -p, pinv) : crt_y(acc[mb][nb][e], p, c16, pinv);
                w[e >> 2] |= y << (8 * (e & 3));
            }
            *(uint4 *)(col.p + (wm * MB + mb) * col.row_bytes + lane * 16) = uint4{w[0], w[1], w[2], w[3]};
        }
        stores += MB;
    }
    return stores;
}

// One 256 x BN output tile of one modulus: the K loop over the plane blocks at gP (left, two
// 128-row blocks tile_stride apart) and gX (right, XSUB 128-column blocks), then the epilogue,
// which stores block column bc at dst(bc) (a wave-uniform CrtBlockCol).
template <class T, class Dst>
__device__ __forceinline__ void crt_tile(int8_t *lds, const int8_t *gP, const int8_t *gX, int KB, int64_t plane_stride,
                                         int p, const Dst &dst) {
    constexpr int MB = T::MB, NB = T::NB, kCrtThreads = T::THREADS, kCrtWavesN = T::WN;
    constexpr int kCrtNbuf = T::NBUF;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave_u / kCrtWavesN, wn = wave_u % kCrtWavesN;
    const int64_t tile_stride = (int64_t)KB * plane_stride;  // bytes of one 128-wide tile

    v16i acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = v16i{0};

    constexpr int CH = kCrtSub / 16;  // 16-byte chunks per block
    // the buffer form of the direct-to-LDS load (byte offsets within a tile's panels stay
    // below 2^32: at most 3 x 2048 k blocks x 16 moduli x 8 KiB)
    const __amdgpu_buffer_rsrc_t rsP = lds_src_rsrc(gP), rsX = lds_src_rsrc(gX);
    auto gload = [&](int kb, int buf) {
        int8_t *dst = lds + buf * T::STAGE;
        const uint32_t off = (uint32_t)kb * (uint32_t)plane_stride;
#pragma unroll
        for (int b = 0; b < 2; ++b)
            copy_to_lds_buf<kCrtThreads, CH>(rsP, (uint32_t)(b * tile_stride) + off, dst + b * kCrtSub, tid, wave_u);
#pragma unroll
        for (int b = 0; b < T::XSUB; ++b)
            copy_to_lds_buf<kCrtThreads, CH>(rsX, (uint32_t)(b * tile_stride) + off, dst + (2 + b) * kCrtSub, tid, wave_u);
    };
    const int loads_per_stage = (2 + T::XSUB) * loads_of_wave<kCrtThreads, CH>(wave_u);

    // plaintext rows of this wave: wm * 32 MB + 32 mb + lane % 32, in 128-row block psub;
    // residue columns: wn * 32 NB + 32 nb + lane % 32, in block (that) / 128
    const int psub = (wm * 32 * MB) / kCrtR;
    const int prow0 = (wm * 32 * MB) % kCrtR;
    struct Frags {
        v4i a[MB], b[NB];
    };
    // the fragments of row block mb / column block nb for K half kk of the stage in buffer buf
    auto frag_a = [&](int buf, int kk, int mb) -> v4i {
        const int8_t *lp = lds + buf * T::STAGE + psub * kCrtSub;
        const int c = kk * 2 + (lane >> 5);
        const int r = prow0 + mb * 32 + (lane & 31);
        return *(const v4i *)(lp + r * 64 + ((c ^ swz(r)) << 4));
    };
    auto frag_b = [&](int buf, int kk, int nb) -> v4i {
        const int8_t *lx = lds + buf * T::STAGE + 2 * kCrtSub;
        const int c = kk * 2 + (lane >> 5);
        const int col = wn * 32 * NB + nb * 32 + (lane & 31);
        const int r = col & (kCrtR - 1);
        return *(const v4i *)(lx + (col / kCrtR) * kCrtSub + r * 64 + ((c ^ swz(r)) << 4));
    };
    // in the order the MFMAs of a half use them (column block by column block)
    auto read_frags = [&](Frags &f, int buf, int kk) {
        f.a[0] = frag_a(buf, kk, 0);
        f.b[0] = frag_b(buf, kk, 0);
        __builtin_amdgcn_sched_barrier(0);  // the first MFMA's two reads go first
#pragma unroll
        for (int mb = 1; mb < MB; ++mb) f.a[mb] = frag_a(buf, kk, mb);
#pragma unroll
        for (int nb = 1; nb < NB; ++nb) f.b[nb] = frag_b(buf, kk, nb);
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
    if constexpr (MB * NB >= 12) {
        // One half-stage of fragments in registers, refilled in place: the MFMAs of a half run
        // column block by column block (nb outer), so b[nb] is dead after its MB MFMAs and each
        // a[mb] after its use in the last column block; each register set is refilled with the
        // next half's fragment as soon as it dies, and the next half starts with the fragments
        // refilled first.  Only the first half after each workgroup barrier waits for all of
        // its reads.  Full groups of G stages run branch-free; a last partial group takes the
        // plain schedule.
        static_assert(G == 2, "four halves per group");
        // the MFMAs of one half from f; with NEXT, refill f from (nbuf, nkk) as registers die
        auto half = [&](Frags &f, bool next, int nbuf, int nkk) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    acc[mb][nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[mb], f.b[nb], acc[mb][nb], 0, 0, 0);
                    if (next) {
                        if (nb < NB - 1 && mb == MB - 1) f.b[nb] = frag_b(nbuf, nkk, nb);
                        if (nb == NB - 1) {
                            f.a[mb] = frag_a(nbuf, nkk, mb);
                            if (mb == MB - 1) f.b[nb] = frag_b(nbuf, nkk, nb);
                        }
                    }
                }
            }
            if (next) {
                // pin the order: MB MFMAs then one read per column block but the last, then
                // one read after each MFMA of the last column block (two after the final one)
#pragma unroll
                for (int nb = 0; nb < NB - 1; ++nb) {
                    __builtin_amdgcn_sched_group_barrier(0x008, MB, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
#pragma unroll
                for (int mb = 0; mb < MB - 1; ++mb) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        };
        const int KBfull = KB - KB % G;
        Frags f;
        settle_scalar_loads();
#pragma unroll 1
        for (int kb = 0; kb < KBfull; kb += G) {
            const int b0 = kb % kCrtNbuf, b1 = (kb + 1) % kCrtNbuf;
            read_frags(f, b0, 0);
            half(f, true, b0, 1);
            half(f, true, b1, 0);
            half(f, true, b1, 1);
            half(f, false, 0, 0);
            wait_lds_after_mfmas();
            wait_vmcnt(outstanding(kb + 2 * G - 1, kb + kCrtNbuf - 1));
            stage_barrier();
#pragma unroll
            for (int h = 0; h < G; ++h)
                if (kb + h + kCrtNbuf < KB) gload(kb + h + kCrtNbuf, (kb + h) % kCrtNbuf);
        }
        if (KBfull < KB) {
            const int cur = KBfull % kCrtNbuf;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                read_frags(f, cur, kk);
                mfmas(f);
            }
        }
    } else {
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
    }

    if (KB <= kCrtShortKB) crt_epilogue<MB, NB, true>(acc, p, wm, wn, lane, dst);
    else crt_epilogue<MB, NB, false>(acc, p, wm, wn, lane, dst);
}

// One output tile of one modulus: its plane blocks (left at gP, two 128-row blocks one
// tile_stride = KB plane_stride apart; right at gX, XSUB 128-column blocks), its K blocks and
// modulus, and where its products go (c0..c2, read by the sequence's dst).
struct CrtRef {
    const int8_t *gP, *gX;
    int KB, p;
    int64_t c0, c1, c2;
};

// The tiles of a persistent workgroup of 256 x 384 tiles, run as one stream of stages through
// the LDS ring: the last groups of a tile load the first stages of the next, so that a tile's
// epilogue and its product-byte stores overlap the next tile's loads and no tile starts with
// an empty pipeline.  Every tile must have an even K-block count of at least NBUF.  The
// workgroup takes its tiles one at a time from a queue; a queue Seq provides
//   uint32_t claim();                  thread 0: start taking the next tile (a returning atomic)
//   int resolve(uint32_t claimed);     thread 0: the tile claimed, or -1 once none is left
//   CrtRef ref(int t) const;           tile t (wave-uniform t)
//   CrtBlockCol dst(const CrtRef &, int bc) const;  where its 32-column block column bc goes
// The claimed index reaches the other waves through LDS, at a barrier where a buffer is free.
template <class T, class Seq>
__device__ __forceinline__ void crt_tiles(int8_t *lds, int64_t plane_stride, Seq &seq) {
    constexpr int MB = T::MB, NB = T::NB, kCrtThreads = T::THREADS, kCrtWavesN = T::WN;
    constexpr int kCrtNbuf = T::NBUF;
    constexpr int G = T::GROUP;
    static_assert(MB * NB >= 12 && G == 2 && kCrtNbuf == 2 * G, "the rolling schedule over a ring of two groups");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave_u / kCrtWavesN, wn = wave_u % kCrtWavesN;

    // the tile index from thread 0 to every wave, through the first bytes of LDS buffer buf
    // (free: no wave reads it and no load into it is in flight)
    auto broadcast = [&](int buf, int t0) -> int {
        int *slot = (int *)(lds + buf * T::STAGE);  // ordered by the barriers' memory clobbers
        if (tid == 0) *slot = t0;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        stage_barrier();
        const int t = __builtin_amdgcn_readfirstlane(*slot);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        stage_barrier();  // every wave has read it before loads overwrite it
        return t;
    };

    v16i acc[MB][NB];
    auto zero_acc = [&]() {
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[a][b] = v16i{0};
    };

    constexpr int CH = kCrtSub / 16;  // 16-byte chunks per block
    // a tile's sources for the buffer form of the direct-to-LDS load, in scalar registers
    // (byte offsets within a tile's panels stay below 2^32: at most 3 x 2048 k blocks x 16
    // moduli x 8 KiB)
    struct Src {
        __amdgpu_buffer_rsrc_t rsP, rsX;
        uint32_t tile_stride;  // bytes of one 128-wide tile
    };
    auto source = [&](const CrtRef &r) -> Src {
        return Src{lds_src_rsrc(r.gP), lds_src_rsrc(r.gX),
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(r.KB * plane_stride))};
    };
    // stage kb of a tile into LDS buffer buf
    auto gload = [&](const Src &src, int kb, int buf) {
        int8_t *dst = lds + buf * T::STAGE;
        const uint32_t off = (uint32_t)kb * (uint32_t)plane_stride;
#pragma unroll
        for (int b = 0; b < 2; ++b)
            copy_to_lds_buf<kCrtThreads, CH>(src.rsP, b * src.tile_stride + off, dst + b * kCrtSub, tid, wave_u);
#pragma unroll
        for (int b = 0; b < T::XSUB; ++b)
            copy_to_lds_buf<kCrtThreads, CH>(src.rsX, b * src.tile_stride + off, dst + (2 + b) * kCrtSub, tid, wave_u);
    };
    const int loads_per_stage = (2 + T::XSUB) * loads_of_wave<kCrtThreads, CH>(wave_u);

    // plaintext rows of this wave: wm * 32 MB + 32 mb + lane % 32, in 128-row block psub;
    // residue columns: wn * 32 NB + 32 nb + lane % 32, in block (that) / 128
    const int psub = (wm * 32 * MB) / kCrtR;
    const int prow0 = (wm * 32 * MB) % kCrtR;
    struct Frags {
        v4i a[MB], b[NB];
    };
    // the fragments of row block mb / column block nb for K half kk of the stage in buffer buf
    auto frag_a = [&](int buf, int kk, int mb) -> v4i {
        const int8_t *lp = lds + buf * T::STAGE + psub * kCrtSub;
        const int c = kk * 2 + (lane >> 5);
        const int r = prow0 + mb * 32 + (lane & 31);
        return *(const v4i *)(lp + r * 64 + ((c ^ swz(r)) << 4));
    };
    auto frag_b = [&](int buf, int kk, int nb) -> v4i {
        const int8_t *lx = lds + buf * T::STAGE + 2 * kCrtSub;
        const int c = kk * 2 + (lane >> 5);
        const int col = wn * 32 * NB + nb * 32 + (lane & 31);
        const int r = col & (kCrtR - 1);
        return *(const v4i *)(lx + (col / kCrtR) * kCrtSub + r * 64 + ((c ^ swz(r)) << 4));
    };
    // in the order the MFMAs of a half use them (column block by column block)
    auto read_frags = [&](Frags &f, int buf, int kk) {
        f.a[0] = frag_a(buf, kk, 0);
        f.b[0] = frag_b(buf, kk, 0);
        __builtin_amdgcn_sched_barrier(0);  // the first MFMA's two reads go first
#pragma unroll
        for (int mb = 1; mb < MB; ++mb) f.a[mb] = frag_a(buf, kk, mb);
#pragma unroll
        for (int nb = 1; nb < NB; ++nb) f.b[nb] = frag_b(buf, kk, nb);
    };

    // the epilogue of tile r; returns the stores issued
    auto epilogue = [&](const CrtRef &r) -> int {
        const auto dst = [&](int bc) { return seq.dst(r, bc); };
        return r.KB <= kCrtShortKB ? crt_epilogue<MB, NB, true>(acc, r.p, wm, wn, lane, dst)
                                   : crt_epilogue<MB, NB, false>(acc, r.p, wm, wn, lane, dst);
    };

    // One half-stage of fragments in registers, refilled in place: the MFMAs of a half run
    // column block by column block (nb outer), so b[nb] is dead after its MB MFMAs and each
    // a[mb] after its use in the last column block; each register set is refilled with the
    // next half's fragment as soon as it dies, and the next half starts with the fragments
    // refilled first.  Only the first half after each workgroup barrier waits for all of its
    // reads.
    auto half = [&](Frags &f, bool next, int nbuf, int nkk) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                acc[mb][nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[mb], f.b[nb], acc[mb][nb], 0, 0, 0);
                if (next) {
                    if (nb < NB - 1 && mb == MB - 1) f.b[nb] = frag_b(nbuf, nkk, nb);
                    if (nb == NB - 1) {
                        f.a[mb] = frag_a(nbuf, nkk, mb);
                        if (mb == MB - 1) f.b[nb] = frag_b(nbuf, nkk, nb);
                    }
                }
            }
        }
        if (next) {
            // pin the order: MB MFMAs then one read per column block but the last, then one
            // read after each MFMA of the last column block (two after the final one)
#pragma unroll
            for (int nb = 0; nb < NB - 1; ++nb) {
                __builtin_amdgcn_sched_group_barrier(0x008, MB, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
#pragma unroll
            for (int mb = 0; mb < MB - 1; ++mb) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    };

    // Stage s of the stream sits in buffer s mod NBUF.  The loads of a group are issued one
    // group ahead of their use, so a group's wait covers every load but those issued since:
    // the last tile's epilogue stores and, at a tile's first wait, the loads of its stages 2
    // and 3.  This rests on vmcnt counting the buffer loads and the epilogue's stores together
    // and retiring them in issue order, as on gfx9 targets, which have no separate store
    // counter.
    int t = broadcast(0, tid == 0 ? seq.resolve(seq.claim()) : 0);
    if (t < 0) return;
    CrtRef cur = seq.ref(t);
    Src cs = source(cur);
#pragma unroll
    for (int st = 0; st < kCrtNbuf; ++st) gload(cs, st, st);
    wait_vmcnt(2 * loads_per_stage);
    stage_barrier();
    int ring = 0, stores = 0;
    Frags f;
#pragma unroll 1
    while (true) {
        // the claim of the next tile goes out now and is read back near the tile's end
        uint32_t claimed = 0;
        if (tid == 0) claimed = seq.claim();
        bool more = false;
        CrtRef nxt = cur;
        Src ns = cs;
        zero_acc();
        const int KB = cur.KB;
        settle_scalar_loads();
        // all groups but the last two: their successors are stages of this tile
#pragma unroll 1
        for (int kb = 0; kb < KB - 2 * G; kb += G) {
            const int b0 = (ring + kb) % kCrtNbuf, b1 = (ring + kb + 1) % kCrtNbuf;
            read_frags(f, b0, 0);
            half(f, true, b0, 1);
            half(f, true, b1, 0);
            half(f, true, b1, 1);
            half(f, false, 0, 0);
            wait_lds_after_mfmas();
            if (kb == 0) wait_vmcnt(stores);
            else wait_vmcnt(0);
            stage_barrier();
#pragma unroll
            for (int h = 0; h < G; ++h) gload(cs, kb + h + kCrtNbuf, (ring + kb + h) % kCrtNbuf);
        }
        // the last two groups: the next tile is learnt, and its first stages loaded
        settle_scalar_loads();
#pragma unroll 1
        for (int kb = KB - 2 * G; kb < KB; kb += G) {
            const int b0 = (ring + kb) % kCrtNbuf, b1 = (ring + kb + 1) % kCrtNbuf;
            read_frags(f, b0, 0);
            half(f, true, b0, 1);
            half(f, true, b1, 0);
            half(f, true, b1, 1);
            half(f, false, 0, 0);
            wait_lds_after_mfmas();
            if (kb + G < KB || more) {
                // the next group's stages have landed: they were issued before the last tile's
                // stores (at a tile's first wait) or are the last loads issued
                if (kb == 0) wait_vmcnt(stores);
                else wait_vmcnt(0);
                stage_barrier();
                if (kb == KB - 2 * G) {
                    // buffers b0, b1 are free: learn the next tile before loading its stages
                    const int tn = broadcast(b0, tid == 0 ? seq.resolve(claimed) : 0);
                    if (tn >= 0) {
                        more = true;
                        nxt = seq.ref(tn);
                        ns = source(nxt);
                    }
                    settle_scalar_loads();
                }
#pragma unroll
                for (int h = 0; h < G; ++h) {
                    const int s = kb + h + kCrtNbuf, buf = (ring + kb + h) % kCrtNbuf;
                    if (s < KB) gload(cs, s, buf);
                    else if (more) gload(ns, s - KB, buf);
                }
            }
        }
        stores = epilogue(cur);
        if (!more) return;
        ring = (ring + KB) % kCrtNbuf;
        cur = nxt;
        cs = ns;
        // the next tile's stages 0 and 1: issued before its stages 2, 3 and the stores
        wait_vmcnt(2 * loads_per_stage + stores);
        stage_barrier();
    }
}

}  // namespace hlb
