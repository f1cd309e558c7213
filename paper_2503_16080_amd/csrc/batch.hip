// batch.hip -- hlb_cp_mm_batch: many CP-MMs of uneven shapes over shared RNS primes.
//
// Every CP-MM is two Mod-PP-MMs per prime (Theorem th:pcmm-shs), and the per-prime products
// are independent (as in Section 6.1, Strategy 3), so a batch is one flat list of output
// tiles.  INT8 form: one launch splits every plaintext, one launch splits every ciphertext
// part, a tiny kernel zeroes the work counter, and one persistent launch (one workgroup per
// CU) pulls tiles from the counter, largest K first.  Each problem uses the tile class the
// planner picks for its shape.  The four launches are captured once per batch signature
// into a HIP graph and replayed on later calls with the same signature.
//
// Multimodular form (Strategy 3): one D for the whole batch (the planner's count for the
// largest K and plaintext bound), one launch splits every left and right operand into its
// residue planes, one GEMM launch covers every (problem, modulus, tile), one launch
// recombines every output matrix; captured and replayed in the same way.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/hlb.h"
#include "common.hpp"
#include "host.hpp"
#include "launch.hpp"
#include "crt.hpp"
#include "crt_jobs.hpp"

namespace hlb {

namespace {

struct BatchLayout {
    int dp = 3, dx = 7;
    bool fold = false;
    int kfold = 0;
    std::vector<SplitJob> pjobs, xjobs;
    int64_t p_wgs = 0, x_wgs = 0;
    std::vector<BatchProb> probs;
    std::vector<BatchSeg> segs;
    int64_t total_items = 0;
    int n_chunks = 1;
    int64_t chunk_begin[kMaxChunks + 1] = {0};
    // workspace offsets (bytes) relative to the workspace base
    size_t off_pjobs = 0, off_xjobs = 0, off_probs = 0, off_segs = 0, off_counter = 0, off_digits = 0;
    size_t off_pmap = 0, off_xmap = 0;  // workgroup -> job maps of the two split launches
    size_t bytes = 0;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Builds descriptors for an INT8 batch.  Digit-buffer pointers are stored as offsets from
// the start of the digit region and rebased by `rebase` once the workspace exists.
hlb_status build_layout(const hlb_cpmm_problem *probs, int count, const uint64_t *primes, int L,
                        BatchLayout &lay) {
    uint64_t qmax = 0;
    for (int l = 0; l < L; ++l) qmax = std::max(qmax, primes[l]);
    Plan base;
    hlb_status st = plan(1, 1, qmax, 1, HLB_FORM_INT8, &base);
    if (st != HLB_OK) return st;
    if (base.np != 3) return HLB_EUNSUP;
    lay.dp = base.np;
    lay.dx = base.nx;
    lay.kfold = (int)std::max<int64_t>(1, base.kchunk / kBK8);

    // problems in descending order of K blocks: longest tiles are handed out first
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].k > probs[b].k; });

    size_t digit_off = 0;
    for (int oi = 0; oi < count; ++oi) {
        const hlb_cpmm_problem &p = probs[order[oi]];
        if (p.m == 0 || p.k == 0 || (p.nA == 0 && p.nB == 0)) continue;
        Plan pl = base;
        choose_class(&pl, p.m, std::max(p.nA, p.nB), p.k);
        const int64_t kblocks = (p.k + kBK8 - 1) / kBK8;
        if (kblocks > lay.kfold) lay.fold = true;
        const int64_t tiles_m = (p.m + pl.bm - 1) / pl.bm;
        const int64_t p_tile = (int64_t)lay.dp * pl.bm * kBK8, x_tile = (int64_t)lay.dx * pl.bn * kBK8;
        // the tiles address their digit panels with 32-bit byte offsets
        if (kblocks * std::max(p_tile, x_tile) > (int64_t)UINT32_MAX) return HLB_EINVAL;

        BatchProb bp;
        std::memset(&bp, 0, sizeof(bp));
        bp.item_start = lay.total_items;
        bp.Pd = (const int8_t *)(uintptr_t)digit_off;
        bp.m = p.m;
        bp.kblocks = (int32_t)kblocks;
        bp.tiles_m = (int32_t)tiles_m;
        bp.cls = pl.cls;
        bp.seg0 = (int32_t)lay.segs.size();

        SplitJob pj;
        std::memset(&pj, 0, sizeof(pj));
        pj.wg_start = lay.p_wgs;
        pj.P = p.P;
        pj.ld = p.ldp;
        pj.rows = p.m;
        pj.k = p.k;
        pj.kblocks = (int32_t)kblocks;
        pj.R = pl.bm;
        pj.rows_side = 1;
        pj.out = (int8_t *)(uintptr_t)digit_off;
        lay.pjobs.push_back(pj);
        lay.p_wgs += tiles_m * kblocks;
        digit_off += (size_t)(tiles_m * kblocks * p_tile);

        bp.Xd = (const int8_t *)(uintptr_t)digit_off;
        int32_t tb = 0;
        for (int l = 0; l < L; ++l) {
            for (int part = 0; part < 2; ++part) {
                const int64_t n = part == 0 ? p.nA : p.nB;
                if (n == 0) continue;
                const uint64_t *X = (part == 0 ? p.A : p.B) + (int64_t)l * p.k * n;
                uint64_t *C = (part == 0 ? p.PA : p.PB) + (int64_t)l * p.m * n;
                const int64_t tiles = (n + pl.bn - 1) / pl.bn;
                BatchSeg sg;
                std::memset(&sg, 0, sizeof(sg));
                sg.C = C;
                sg.ldc = n;
                sg.n = n;
                sg.q = primes[l];
                sg.qinv = 1.0 / (double)primes[l];
                sg.tile_begin = tb;
                lay.segs.push_back(sg);
                SplitJob xj;
                std::memset(&xj, 0, sizeof(xj));
                xj.wg_start = lay.x_wgs;
                xj.X = X;
                xj.ld = n;
                xj.cols = n;
                xj.k = p.k;
                xj.kblocks = (int32_t)kblocks;
                xj.R = pl.bn;
                xj.rows_side = 0;
                xj.out = (int8_t *)(uintptr_t)(digit_off + (size_t)tb * kblocks * x_tile);
                lay.xjobs.push_back(xj);
                lay.x_wgs += tiles * kblocks;
                tb += (int32_t)tiles;
            }
        }
        bp.tiles_n = tb;
        bp.nseg = (int32_t)lay.segs.size() - bp.seg0;
        digit_off += (size_t)tb * kblocks * x_tile;
        lay.total_items += tiles_m * tb;
        lay.probs.push_back(bp);
    }
    if (lay.total_items > INT32_MAX || lay.p_wgs > INT32_MAX || lay.x_wgs > INT32_MAX) return HLB_EINVAL;
    // cut the work list into n_chunks contiguous chunks of about equal cost (a tile costs
    // its K blocks plus about two blocks of prologue and epilogue)
    int n_xcd = 8;
    (void)device_ready(&n_xcd);
    lay.n_chunks = std::max(1, std::min(n_xcd, kMaxChunks));
    double total_cost = 0.0;
    for (const BatchProb &bp : lay.probs) total_cost += (double)bp.tiles_m * bp.tiles_n * (bp.kblocks + 2);
    int c = 1;
    double acc = 0.0;  // cost of all items before the current problem
    for (const BatchProb &bp : lay.probs) {
        const double per = bp.kblocks + 2.0;
        const int64_t items = (int64_t)bp.tiles_m * bp.tiles_n;
        // every cut whose target cost falls inside this problem
        while (c < lay.n_chunks && acc + items * per >= total_cost * c / lay.n_chunks) {
            const double need = total_cost * c / lay.n_chunks - acc;
            const int64_t i = std::min<int64_t>(items, std::max<int64_t>(0, (int64_t)std::ceil(need / per)));
            lay.chunk_begin[c++] = bp.item_start + i;
        }
        acc += items * per;
    }
    for (; c <= lay.n_chunks; ++c) lay.chunk_begin[c] = lay.total_items;
    lay.chunk_begin[lay.n_chunks] = lay.total_items;
    size_t off = 0;
    lay.off_pjobs = off;
    off = align_up(off + lay.pjobs.size() * sizeof(SplitJob), 256);
    lay.off_xjobs = off;
    off = align_up(off + lay.xjobs.size() * sizeof(SplitJob), 256);
    lay.off_probs = off;
    off = align_up(off + lay.probs.size() * sizeof(BatchProb), 256);
    lay.off_segs = off;
    off = align_up(off + lay.segs.size() * sizeof(BatchSeg), 256);
    lay.off_counter = off;
    off = align_up(off + 256, 256);
    lay.off_pmap = off;
    off = align_up(off + (size_t)lay.p_wgs * sizeof(int32_t), 256);
    lay.off_xmap = off;
    off = align_up(off + (size_t)lay.x_wgs * sizeof(int32_t), 256);
    lay.off_digits = off;
    lay.bytes = off + digit_off;
    return HLB_OK;
}

// Turns digit offsets into device addresses inside a workspace at `base`.
void rebase(BatchLayout &lay, char *base) {
    char *digits = base + lay.off_digits;
    for (SplitJob &j : lay.pjobs) j.out = (int8_t *)(digits + (uintptr_t)j.out);
    for (SplitJob &j : lay.xjobs) j.out = (int8_t *)(digits + (uintptr_t)j.out);
    for (BatchProb &p : lay.probs) {
        p.Pd = (const int8_t *)(digits + (uintptr_t)p.Pd);
        p.Xd = (const int8_t *)(digits + (uintptr_t)p.Xd);
    }
}

// Host image of the descriptor region (everything before the digit buffers).
std::vector<char> descriptor_image(const BatchLayout &lay) {
    std::vector<char> img(lay.off_digits, 0);
    std::memcpy(img.data() + lay.off_pjobs, lay.pjobs.data(), lay.pjobs.size() * sizeof(SplitJob));
    std::memcpy(img.data() + lay.off_xjobs, lay.xjobs.data(), lay.xjobs.size() * sizeof(SplitJob));
    std::memcpy(img.data() + lay.off_probs, lay.probs.data(), lay.probs.size() * sizeof(BatchProb));
    std::memcpy(img.data() + lay.off_segs, lay.segs.data(), lay.segs.size() * sizeof(BatchSeg));
    // job j owns workgroups [wg_start_j, wg_start_{j+1}), the last job up to `total`
    auto fill_map = [&](const std::vector<SplitJob> &jobs, size_t off, int64_t total) {
        int32_t *map = (int32_t *)(img.data() + off);
        for (size_t j = 0; j < jobs.size(); ++j) {
            const int64_t stop = j + 1 < jobs.size() ? jobs[j + 1].wg_start : total;
            for (int64_t w = jobs[j].wg_start; w < stop; ++w) map[w] = (int32_t)j;
        }
    };
    fill_map(lay.pjobs, lay.off_pmap, lay.p_wgs);
    fill_map(lay.xjobs, lay.off_xmap, lay.x_wgs);
    return img;
}

// The launch sequence of a batch on stream s (capturable: kernels only).
hlb_status enqueue(const BatchLayout &lay, char *base, int grid, hipStream_t s) {
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.probs = (const BatchProb *)(base + lay.off_probs);
    a.segs = (const BatchSeg *)(base + lay.off_segs);
    a.counters = (unsigned int *)(base + lay.off_counter);
    a.total_items = lay.total_items;
    a.n_chunks = lay.n_chunks;
    for (int i = 0; i <= lay.n_chunks; ++i) a.chunk_begin[i] = lay.chunk_begin[i];
    a.nprob = (int32_t)lay.probs.size();
    a.kfold = lay.fold ? lay.kfold : INT32_MAX;
    a.group_m = 4;
    {
        ProfScope ps("split_p", s);
        if (launch_split_batch_i8(lay.dp, (const SplitJob *)(base + lay.off_pjobs),
                                  (const int32_t *)(base + lay.off_pmap), lay.p_wgs, s) != hipSuccess)
            return HLB_EDEVICE;
    }
    {
        ProfScope ps("split_x", s);
        if (launch_split_batch_i8(lay.dx, (const SplitJob *)(base + lay.off_xjobs),
                                  (const int32_t *)(base + lay.off_xmap), lay.x_wgs, s) != hipSuccess)
            return HLB_EDEVICE;
    }
    if (launch_reset_counter(a.counters, s) != hipSuccess) return HLB_EDEVICE;
    ProfScope ps("batch_i8", s);
    if (launch_gemm_i8_batch(lay.dp, lay.dx, lay.fold, a, grid, s) != hipSuccess) return HLB_EDEVICE;
    return HLB_OK;
}


// ------------------------------- multimodular batch -------------------------------------
// Marks, before rebasing, a batch GEMM tile's plane tile that lies past its problem's outputs.
constexpr uintptr_t kNoPlane = ~(uintptr_t)0;

// The GEMM items of one tile class: their own persistent launch, runs and queue counters.
struct CrtClassItems {
    std::vector<CrtItem> items;
    int64_t chunk[kMaxChunks + 1] = {0};
    size_t off_items = 0, off_counters = 0;
};

struct CrtBatchLayout {
    int D = 0;
    CrtScale scale;
    std::vector<CrtSplitJob> sjobs;
    int64_t split_wgs = 0;
    CrtClassItems cls[kCrtClasses];
    std::vector<int> prob_cls;  // tile class of every non-empty problem, in problem order
    int n_chunks = 1;
    std::vector<CrtSeg> segs;
    std::vector<CrtCombineJob> cjobs;
    int64_t combine_wgs = 0;
    int64_t total_items = 0;
    // descriptor offsets, then the residue planes (offsets relative to off_planes) and the
    // product planes (offsets relative to off_ybytes)
    size_t off_sjobs = 0, off_cjobs = 0, off_planes = 0, off_ybytes = 0, bytes = 0;
};

hlb_status build_crt_layout(const hlb_cpmm_problem *probs, int count, const uint64_t *primes, int L,
                            CrtBatchLayout &lay) {
    uint64_t qmax = 0;
    for (int l = 0; l < L; ++l) qmax = std::max(qmax, primes[l]);
    int64_t kmax = 1, pmax = 1;
    for (int i = 0; i < count; ++i) {
        const hlb_cpmm_problem &p = probs[i];
        if (p.m == 0 || p.k == 0 || (p.nA == 0 && p.nB == 0)) continue;
        kmax = std::max(kmax, p.k);
        pmax = std::max(pmax, p.p_absmax);
    }
    Plan pl;
    pl.kind = 1;
    hlb_status st = plan(1, kmax, qmax, pmax, HLB_FORM_INT8_CRT, &pl);
    if (st != HLB_OK) return st;
    const int D = pl.np;
    lay.D = D;
    unsigned __int128 M = 1;
    for (int i = 0; i < D; ++i) M *= (unsigned)kCrtModuli[i];
    std::memset(&lay.scale, 0, sizeof(lay.scale));
    for (int i = 0; i < D; ++i) {
        const int p = kCrtModuli[i];
        const int mi = (int)((M / (unsigned)p) % (unsigned)p);
        for (int v = 1; v < p; ++v)
            if ((mi * v) % p == 1) {
                lay.scale.s[i] = v;
                break;
            }
    }

    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].k > probs[b].k; });
    const int64_t sub = (int64_t)D * 128 * kBK8;  // bytes of one 128-wide tile and k block
    // every problem's GEMM tile class (tuning table, or the forced class)
    std::vector<int> pcls(count, -1);
    for (int i = 0; i < count; ++i) {
        const hlb_cpmm_problem &p = probs[i];
        if (p.m == 0 || p.k == 0 || (p.nA == 0 && p.nB == 0)) continue;
        pcls[i] = crt_tile_class(D, p.m, std::max(p.nA, p.nB), p.k);
        lay.prob_cls.push_back(pcls[i]);
    }
    size_t plane_off = 0, y_off = 0;
    for (int oi = 0; oi < count; ++oi) {
        const hlb_cpmm_problem &p = probs[order[oi]];
        if (p.m == 0 || p.k == 0 || (p.nA == 0 && p.nB == 0)) continue;
        CrtClassItems &ci = lay.cls[pcls[order[oi]]];
        const int64_t xsub = crt_tile_cols(pcls[order[oi]]) / 128;
        const int64_t kblocks = (p.k + kBK8 - 1) / kBK8;
        const int64_t lt = ((p.m + 255) / 256) * 2, tiles_m = lt / 2;

        CrtSplitJob pj;
        std::memset(&pj, 0, sizeof(pj));
        pj.wg_start = lay.split_wgs;
        pj.src = p.P;
        pj.ld = p.ldp;
        pj.extent = p.m;
        pj.k = p.k;
        pj.qc = 0;
        pj.kblocks = (int32_t)kblocks;
        pj.rows_side = 1;
        pj.out = (int8_t *)(uintptr_t)plane_off;
        lay.sjobs.push_back(pj);
        lay.split_wgs += lt * kblocks;
        plane_off += (size_t)(lt * kblocks * sub);

        const size_t p_off = (size_t)(uintptr_t)pj.out, x_off = plane_off;
        const size_t seg0 = lay.segs.size();
        // the problem's output matrices lie side by side in 128-column plane tiles
        int64_t tb = 0;
        for (int l = 0; l < L; ++l) {
            for (int part = 0; part < 2; ++part) {
                const int64_t n = part == 0 ? p.nA : p.nB;
                if (n == 0) continue;
                const uint64_t *X = (part == 0 ? p.A : p.B) + (int64_t)l * p.k * n;
                uint64_t *C = (part == 0 ? p.PA : p.PB) + (int64_t)l * p.m * n;
                const int64_t t128 = (n + 127) / 128;
                CrtSplitJob xj;
                std::memset(&xj, 0, sizeof(xj));
                xj.wg_start = lay.split_wgs;
                xj.src = X;
                xj.ld = n;
                xj.extent = n;
                xj.k = p.k;
                xj.qc = primes[l];
                xj.kblocks = (int32_t)kblocks;
                xj.rows_side = 0;
                xj.out = (int8_t *)(uintptr_t)(plane_off + (size_t)(tb * kblocks * sub));
                lay.sjobs.push_back(xj);
                lay.split_wgs += t128 * kblocks;

                CrtSeg sg;
                std::memset(&sg, 0, sizeof(sg));
                sg.Y = (uint8_t *)(uintptr_t)y_off;
                sg.n = n;
                sg.nbc = t128 * 4;
                sg.plane = (tiles_m * 256) * (t128 * 128);
                sg.tile_begin = (int32_t)tb;
                sg.tiles = (int32_t)t128;
                lay.segs.push_back(sg);

                CrtCombineJob cj;
                std::memset(&cj, 0, sizeof(cj));
                cj.wg_start = lay.combine_wgs;
                CrtCombineArgs &c = cj.a;
                c.Y = sg.Y;
                c.C = C;
                c.m = p.m;
                c.n = n;
                c.nbc = sg.nbc;
                c.plane = sg.plane;
                c.ldc = n;
                c.q = primes[l];
                c.barrett = (uint64_t)((~(unsigned __int128)0 >> 64) / c.q);
                c.Mq = (uint64_t)(M % c.q);
                c.D = D;
                for (int j = 0; j < D; ++j) c.w[j] = (uint64_t)((M / (unsigned)kCrtModuli[j]) % c.q);
                lay.cjobs.push_back(cj);
                lay.combine_wgs += crt_combine_wgs(p.m, n);
                y_off += (size_t)(D * sg.plane);
                tb += t128;
            }
        }
        // GEMM tiles are xsub plane tiles wide; the last may reach xsub - 1 plane tiles past the
        // problem's, so those are reserved too (never written, read only for discarded columns)
        const int64_t tg = (tb + xsub - 1) / xsub;
        plane_off += (size_t)((tb + xsub - 1) * kblocks * sub);
        const int64_t items = (int64_t)D * tiles_m * tg;
        if (lay.total_items + items > INT32_MAX) return HLB_EINVAL;
        // the problem's tiles, modulus by modulus (tiles of different moduli share no operand
        // bytes), each modulus's tiles_m x tg grid walked group_m row tiles at a time, column
        // by column (neighbours share operand panels; measured 1.7 % faster on the 64-problem
        // batch than groups of 4 row bands across moduli); offsets are rebased once the
        // workspace exists (kNoPlane marks a plane tile past the problem's outputs)
        const int64_t tile_stride = kblocks * sub, group_m = 8;
        for (int64_t local = 0; local < items; ++local) {
            const int64_t per_mod = tiles_m * tg, mi = local / per_mod, lm = local % per_mod;
            const int64_t span = group_m * tg, gi = lm / span, first = gi * group_m;
            const int64_t gm = std::min(group_m, tiles_m - first), in = lm - gi * span;
            const int64_t rb = first + in % gm, cb = in / gm;
            CrtItem it;
            std::memset(&it, 0, sizeof(it));
            it.P = (const int8_t *)(uintptr_t)(p_off + (size_t)(2 * rb * tile_stride + mi * 128 * kBK8));
            it.X = (const int8_t *)(uintptr_t)(x_off + (size_t)(cb * xsub * tile_stride + mi * 128 * kBK8));
            for (int j = 0; j < kCrtItemCols; ++j) {
                const int64_t pt = cb * xsub + j;
                it.Y[j] = (uint8_t *)kNoPlane;
                for (size_t si = seg0; si < lay.segs.size(); ++si) {
                    const CrtSeg &sg = lay.segs[si];
                    if (pt < sg.tile_begin || pt >= sg.tile_begin + sg.tiles) continue;
                    it.Y[j] = (uint8_t *)(uintptr_t)((uintptr_t)sg.Y + (size_t)(mi * sg.plane));
                    it.nbc[j] = sg.nbc;
                    it.bct[j] = (int32_t)((pt - sg.tile_begin) * 4);
                    break;
                }
            }
            it.kblocks = (int32_t)kblocks;
            it.p = kCrtModuli[mi];
            it.brt = (int32_t)(rb * 8);
            ci.items.push_back(it);
        }
        lay.total_items += items;
    }
    if (lay.total_items > INT32_MAX || lay.split_wgs > INT32_MAX || lay.combine_wgs > INT32_MAX) return HLB_EINVAL;
    // per class, one contiguous run of items per XCD, of about equal cost: an item costs its K
    // blocks plus a fixed cost worth about twelve of them (pipeline fill, epilogue, launch;
    // measured on the 64-problem batch: 2, 8, 12, 20 -> 22.8, 18.3, 16.2, 17.2 ms for the GEMM)
    int n_xcd = 8;
    (void)device_ready(&n_xcd);
    lay.n_chunks = std::max(1, std::min(n_xcd, kMaxChunks));
    constexpr double kItemFixed = 12.0;
    for (CrtClassItems &ci : lay.cls) {
        const int64_t n_items = (int64_t)ci.items.size();
        double total_cost = 0.0;
        for (const CrtItem &it : ci.items) total_cost += it.kblocks + kItemFixed;
        int c = 1;
        double acc = 0.0;
        for (int64_t i = 0; i < n_items && c < lay.n_chunks; ++i) {
            acc += ci.items[i].kblocks + kItemFixed;
            while (c < lay.n_chunks && acc >= total_cost * c / lay.n_chunks) ci.chunk[c++] = i + 1;
        }
        for (; c <= lay.n_chunks; ++c) ci.chunk[c] = n_items;
        ci.chunk[0] = 0;
        ci.chunk[lay.n_chunks] = n_items;
    }
    size_t off = 0;
    lay.off_sjobs = off;
    off = align_up(off + lay.sjobs.size() * sizeof(CrtSplitJob), 256);
    for (CrtClassItems &ci : lay.cls) {
        ci.off_items = off;
        off = align_up(off + ci.items.size() * sizeof(CrtItem), 256);
        ci.off_counters = off;
        off = align_up(off + kMaxChunks * sizeof(unsigned int), 256);
    }
    lay.off_cjobs = off;
    off = align_up(off + lay.cjobs.size() * sizeof(CrtCombineJob), 256);
    lay.off_planes = off;
    lay.off_ybytes = align_up(off + plane_off, 256);
    lay.bytes = lay.off_ybytes + y_off;
    return HLB_OK;
}

// Turns plane offsets into device addresses inside a workspace at `base`.
void rebase_crt(CrtBatchLayout &lay, char *base) {
    char *planes = base + lay.off_planes, *ybytes = base + lay.off_ybytes;
    for (CrtSplitJob &j : lay.sjobs) j.out = (int8_t *)(planes + (uintptr_t)j.out);
    for (CrtClassItems &ci : lay.cls)
        for (CrtItem &it : ci.items) {
            it.P = (const int8_t *)(planes + (uintptr_t)it.P);
            it.X = (const int8_t *)(planes + (uintptr_t)it.X);
            for (int j = 0; j < kCrtItemCols; ++j)
                it.Y[j] = (uintptr_t)it.Y[j] == kNoPlane ? nullptr : (uint8_t *)(ybytes + (uintptr_t)it.Y[j]);
        }
    for (CrtCombineJob &j : lay.cjobs) j.a.Y = (const uint8_t *)(ybytes + (uintptr_t)j.a.Y);
}

std::vector<char> crt_descriptor_image(const CrtBatchLayout &lay) {
    std::vector<char> img(lay.off_planes, 0);
    std::memcpy(img.data() + lay.off_sjobs, lay.sjobs.data(), lay.sjobs.size() * sizeof(CrtSplitJob));
    for (const CrtClassItems &ci : lay.cls)
        std::memcpy(img.data() + ci.off_items, ci.items.data(), ci.items.size() * sizeof(CrtItem));
    std::memcpy(img.data() + lay.off_cjobs, lay.cjobs.data(), lay.cjobs.size() * sizeof(CrtCombineJob));
    return img;
}

// The launches of a multimodular batch on stream s (capturable: kernels only): the split,
// one persistent GEMM per tile class present, the recombination.
hlb_status enqueue_crt(const CrtBatchLayout &lay, char *base, hipStream_t s) {
    {
        ProfScope ps("crt_split_batch", s);
        if (launch_crt_split_batch(lay.D, (const CrtSplitJob *)(base + lay.off_sjobs), (int)lay.sjobs.size(),
                                   lay.split_wgs, lay.scale, s) != hipSuccess)
            return HLB_EDEVICE;
    }
    int n_xcd = 8, cus = 256;
    (void)device_ready(&n_xcd, &cus);
    for (int c = kCrtClasses - 1; c >= 0; --c) {
        const CrtClassItems &ci = lay.cls[c];
        if (ci.items.empty()) continue;
        CrtBatchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.items = (const CrtItem *)(base + ci.off_items);
        a.counters = (unsigned int *)(base + ci.off_counters);
        a.total_items = (int64_t)ci.items.size();
        a.D = lay.D;
        a.n_xcd = lay.n_chunks;
        for (int x = 0; x <= lay.n_chunks; ++x) a.chunk[x] = ci.chunk[x];
        if (launch_reset_counter(a.counters, s) != hipSuccess) return HLB_EDEVICE;
        ProfScope ps("crt_gemm_batch", s);
        if (launch_crt_gemm_batch(c, a, cus, s) != hipSuccess) return HLB_EDEVICE;
    }
    ProfScope ps("crt_combine_batch", s);
    if (launch_crt_combine_batch((const CrtCombineJob *)(base + lay.off_cjobs), (int)lay.cjobs.size(), lay.combine_wgs,
                                 s) != hipSuccess)
        return HLB_EDEVICE;
    return HLB_OK;
}

// ------------------------------- graph cache -------------------------------------------
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char *ws = nullptr;
};
std::mutex g_graph_mu;
std::map<std::vector<uint64_t>, GraphEntry> g_graphs;
constexpr size_t kMaxGraphs = 16;

void destroy_entry(GraphEntry &e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    if (e.ws) (void)hipFree(e.ws);
    e = GraphEntry{};
}

// Everything the captured launches depend on: device, stream, every problem field, the
// primes, and the plan (digit counts, fold chunk, tile class of every problem).
std::vector<uint64_t> signature(const hlb_cpmm_problem *probs, int count, const uint64_t *primes, int L,
                                int dev, hipStream_t s, const BatchLayout &lay) {
    std::vector<uint64_t> sig;
    sig.reserve((size_t)count * 11 + L + lay.probs.size() + 8);
    sig.push_back((uint64_t)dev);
    sig.push_back((uint64_t)(uintptr_t)s);
    sig.push_back((uint64_t)lay.dp);
    sig.push_back((uint64_t)lay.dx);
    sig.push_back((uint64_t)(lay.fold ? lay.kfold : 0));
    sig.push_back((uint64_t)lay.n_chunks);
    for (const BatchProb &p : lay.probs) sig.push_back((uint64_t)p.cls);
    sig.push_back((uint64_t)L);
    for (int l = 0; l < L; ++l) sig.push_back(primes[l]);
    for (int i = 0; i < count; ++i) {
        const hlb_cpmm_problem &p = probs[i];
        const uint64_t f[] = {(uint64_t)p.m, (uint64_t)p.k, (uint64_t)p.nA, (uint64_t)p.nB, (uint64_t)(uintptr_t)p.P,
                              (uint64_t)p.ldp, (uint64_t)p.p_absmax, (uint64_t)(uintptr_t)p.A,
                              (uint64_t)(uintptr_t)p.B, (uint64_t)(uintptr_t)p.PA, (uint64_t)(uintptr_t)p.PB};
        sig.insert(sig.end(), f, f + 11);
    }
    return sig;
}

// Key of a cached multimodular batch graph: a tag, device, stream, D, every problem's tile
// class, the primes and every problem field.
std::vector<uint64_t> crt_signature(const hlb_cpmm_problem *probs, int count, const uint64_t *primes, int L, int dev,
                                    hipStream_t s, int D, const std::vector<int> &prob_cls) {
    std::vector<uint64_t> sig;
    sig.reserve((size_t)count * 11 + L + 8);
    sig.push_back(0x4352544241544348ull);  // distinguishes these keys from the digit batch's
    sig.push_back((uint64_t)dev);
    sig.push_back((uint64_t)(uintptr_t)s);
    sig.push_back((uint64_t)D);
    for (int c : prob_cls) sig.push_back((uint64_t)c);
    sig.push_back((uint64_t)L);
    for (int l = 0; l < L; ++l) sig.push_back(primes[l]);
    for (int i = 0; i < count; ++i) {
        const hlb_cpmm_problem &p = probs[i];
        const uint64_t f[] = {(uint64_t)p.m, (uint64_t)p.k, (uint64_t)p.nA, (uint64_t)p.nB, (uint64_t)(uintptr_t)p.P,
                              (uint64_t)p.ldp, (uint64_t)p.p_absmax, (uint64_t)(uintptr_t)p.A,
                              (uint64_t)(uintptr_t)p.B, (uint64_t)(uintptr_t)p.PA, (uint64_t)(uintptr_t)p.PB};
        sig.insert(sig.end(), f, f + 11);
    }
    return sig;
}

// A multimodular batch: eager (stream-ordered workspace, descriptors uploaded, three
// launches), or captured once per signature into a cached graph with its own workspace.
hlb_status run_crt_batch(const hlb_cpmm_problem *probs, int count, const uint64_t *primes, int L, hipStream_t s) {
    CrtBatchLayout lay;
    hlb_status st = build_crt_layout(probs, count, primes, L, lay);
    if (st != HLB_OK) return st;
    if (lay.total_items == 0) return HLB_OK;
    if (!opt_batch_graph()) {
        void *ws = nullptr;
        WsLease lease;
        const size_t bytes = lay.bytes;
        if ((st = lease.take(s, &bytes, &ws, 1)) != HLB_OK) return st;
        rebase_crt(lay, (char *)ws);
        std::vector<char> img = crt_descriptor_image(lay);
        if (hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, s) != hipSuccess) st = HLB_EDEVICE;
        if (st == HLB_OK) st = enqueue_crt(lay, (char *)ws, s);
        // the host image must outlive the copy
        if (hipStreamSynchronize(s) != hipSuccess && st == HLB_OK) st = HLB_EDEVICE;
        // the lease returns the workspace block to the stream
        return st;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    const std::vector<uint64_t> sig = crt_signature(probs, count, primes, L, dev, s, lay.D, lay.prob_cls);
    std::lock_guard<std::mutex> g(g_graph_mu);
    auto it = g_graphs.find(sig);
    if (it == g_graphs.end()) {
        if (g_graphs.size() >= kMaxGraphs) {
            if (hipStreamSynchronize(s) != hipSuccess) return HLB_EDEVICE;
            for (auto &kv : g_graphs) destroy_entry(kv.second);
            g_graphs.clear();
        }
        GraphEntry e;
        if (hipMalloc((void **)&e.ws, lay.bytes) != hipSuccess) {
            (void)hipGetLastError();
            return HLB_ENOMEM;
        }
        rebase_crt(lay, e.ws);
        std::vector<char> img = crt_descriptor_image(lay);
        if (hipMemcpy(e.ws, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) {
            destroy_entry(e);
            return HLB_EDEVICE;
        }
        hipStream_t cap = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            destroy_entry(e);
            return HLB_EDEVICE;
        }
        hlb_status cst = HLB_OK;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) cst = HLB_EDEVICE;
        if (cst == HLB_OK) {
            cst = enqueue_crt(lay, e.ws, cap);
            if (hipStreamEndCapture(cap, &e.graph) != hipSuccess && cst == HLB_OK) cst = HLB_EDEVICE;
        }
        (void)hipStreamDestroy(cap);
        if (cst == HLB_OK && hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess)
            cst = HLB_EDEVICE;
        if (cst != HLB_OK) {
            (void)hipGetLastError();
            destroy_entry(e);
            return cst;
        }
        it = g_graphs.emplace(sig, e).first;
    }
    return hipGraphLaunch(it->second.exec, s) == hipSuccess ? HLB_OK : HLB_EDEVICE;
}

int persistent_grid(const BatchLayout &lay) {
    int n_xcd = 8, cus = 256;
    (void)device_ready(&n_xcd, &cus);  // cached per device
    return (int)std::min<int64_t>(cus, lay.total_items);
}

}  // namespace

void batch_release() {
    std::lock_guard<std::mutex> g(g_graph_mu);
    for (auto &kv : g_graphs) destroy_entry(kv.second);
    g_graphs.clear();
}

}  // namespace hlb

using namespace hlb;

extern "C" hlb_status hlb_cp_mm_batch(const hlb_cpmm_problem *probs, int count, const uint64_t *primes, int L,
                                      int form, void *stream) {
    if (count < 0 || (count > 0 && !probs) || L < 0 || L > 1024 || (L > 0 && !primes)) return HLB_EINVAL;
    if (count == 0 || L == 0) return HLB_OK;
    for (int l = 0; l < L; ++l)
        if (check_modulus(primes[l]) != HLB_OK) return HLB_EINVAL;
    // argument checks for every problem before any work is enqueued
    for (int i = 0; i < count; ++i) {
        const hlb_cpmm_problem &p = probs[i];
        if (p.m < 0 || p.k < 0 || p.nA < 0 || p.nB < 0 || p.p_absmax < 0 || (uint64_t)p.p_absmax >= kMaxModulus)
            return HLB_EINVAL;
        if (p.m == 0 || (p.nA == 0 && p.nB == 0)) continue;
        if ((p.nA > 0 && !p.PA) || (p.nB > 0 && !p.PB)) return HLB_EINVAL;
        if (p.k > 0 && (!p.P || p.ldp < p.k || (p.nA > 0 && !p.A) || (p.nB > 0 && !p.B))) return HLB_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    hlb_status st = device_ready(nullptr);
    if (st != HLB_OK) return st;
    form = resolve_form(form);
    if (opt_validate()) {
        for (int i = 0; i < count; ++i) {
            const hlb_cpmm_problem &p = probs[i];
            st = validate_cp_mm(p.m, p.k, p.nA, p.nB, p.P, p.ldp, p.p_absmax, p.A, p.B, primes, L, stream);
            if (st != HLB_OK) return st;
        }
    }

    // The persistent INT8 path needs every plaintext within 3 digits; other batches (and the
    // FP64 form) run problem by problem through hlb_cp_mm.
    bool persistent = form == HLB_FORM_INT8 || form == HLB_FORM_AUTO;
    std::vector<hlb_cpmm_problem> local(probs, probs + count);
    for (hlb_cpmm_problem &p : local) {
        if (p.m == 0 || p.k == 0 || (p.nA == 0 && p.nB == 0)) continue;
        if (p.p_absmax == 0) {
            int64_t mx = 0;
            if ((st = hlb_plaintext_absmax(p.P, p.m, p.k, p.ldp, &mx, stream)) != HLB_OK) return st;
            if ((uint64_t)mx >= kMaxModulus) return HLB_ERANGE;
            p.p_absmax = std::max<int64_t>(mx, 1);
        }
        if (i8_digits_for((uint64_t)p.p_absmax) > 3) persistent = false;
    }
    uint64_t qmax = 0;
    for (int l = 0; l < L; ++l) qmax = std::max(qmax, primes[l]);
    if (i8_digits_for(qmax - 1) > 7) persistent = false;
    const bool multimodular = form == HLB_FORM_INT8_CRT;
    if (!persistent && !multimodular) {
        for (const hlb_cpmm_problem &p : local) {
            st = hlb_cp_mm(p.m, p.k, p.nA, p.nB, p.P, p.ldp, p.p_absmax, p.A, p.B, primes, L, p.PA, p.PB, form, stream);
            if (st != HLB_OK) return st;
        }
        return HLB_OK;
    }
    // k == 0 problems write zeros; they take no tiles
    for (const hlb_cpmm_problem &p : local) {
        if (p.k != 0 || p.m == 0) continue;
        for (int l = 0; l < L; ++l) {
            if (launch_zero(p.PA + (int64_t)l * p.m * p.nA, p.m, p.nA, p.nA, s) != hipSuccess ||
                launch_zero(p.PB + (int64_t)l * p.m * p.nB, p.m, p.nB, p.nB, s) != hipSuccess)
                return HLB_EDEVICE;
        }
    }

    if (multimodular) return run_crt_batch(local.data(), count, primes, L, s);
    BatchLayout lay;
    if ((st = build_layout(local.data(), count, primes, L, lay)) != HLB_OK) return st;
    if (lay.total_items == 0) return HLB_OK;
    const int grid = persistent_grid(lay);

    if (!opt_batch_graph()) {
        // eager: stream-ordered workspace, descriptors uploaded, four launches
        void *ws = nullptr;
        WsLease lease;
        const size_t bytes = lay.bytes;
        if ((st = lease.take(s, &bytes, &ws, 1)) != HLB_OK) return st;
        rebase(lay, (char *)ws);
        std::vector<char> img = descriptor_image(lay);
        if (hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, s) != hipSuccess) st = HLB_EDEVICE;
        if (st == HLB_OK) st = enqueue(lay, (char *)ws, grid, s);
        // the host image must outlive the copy
        if (hipStreamSynchronize(s) != hipSuccess && st == HLB_OK) st = HLB_EDEVICE;
        // the lease returns the workspace block to the stream
        return st;
    }

    int dev = 0;
    (void)hipGetDevice(&dev);
    const std::vector<uint64_t> sig = signature(local.data(), count, primes, L, dev, s, lay);
    std::lock_guard<std::mutex> g(g_graph_mu);
    auto it = g_graphs.find(sig);
    if (it == g_graphs.end()) {
        if (g_graphs.size() >= kMaxGraphs) {
            // keep the cache bounded: drop everything (entries are cheap to rebuild)
            if (hipStreamSynchronize(s) != hipSuccess) return HLB_EDEVICE;
            for (auto &kv : g_graphs) destroy_entry(kv.second);
            g_graphs.clear();
        }
        GraphEntry e;
        if (hipMalloc((void **)&e.ws, lay.bytes) != hipSuccess) {
            (void)hipGetLastError();
            return HLB_ENOMEM;
        }
        rebase(lay, e.ws);
        std::vector<char> img = descriptor_image(lay);
        if (hipMemcpy(e.ws, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) {
            destroy_entry(e);
            return HLB_EDEVICE;
        }
        hipStream_t cap = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            destroy_entry(e);
            return HLB_EDEVICE;
        }
        hlb_status cst = HLB_OK;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) cst = HLB_EDEVICE;
        if (cst == HLB_OK) {
            cst = enqueue(lay, e.ws, grid, cap);
            if (hipStreamEndCapture(cap, &e.graph) != hipSuccess && cst == HLB_OK) cst = HLB_EDEVICE;
        }
        (void)hipStreamDestroy(cap);
        if (cst == HLB_OK && hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess)
            cst = HLB_EDEVICE;
        if (cst != HLB_OK) {
            (void)hipGetLastError();
            destroy_entry(e);
            return cst;
        }
        it = g_graphs.emplace(sig, e).first;
    }
    return hipGraphLaunch(it->second.exec, s) == hipSuccess ? HLB_OK : HLB_EDEVICE;
}
