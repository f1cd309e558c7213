// api.cpp -- libhlb host side: argument checks, the exact limb planner, workspace, kernel
// dispatch and the extern "C" entry points declared in include/hlb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hlb.h"
#include "common.hpp"
#include "launch.hpp"
#include "host.hpp"
#include "crt.hpp"
#include "crt_jobs.hpp"

namespace hlb {

// ---------------------------------------------------------------------------------------
// Options and profiling
// ---------------------------------------------------------------------------------------
static std::atomic<int64_t> g_force_kchunk{0};
static std::atomic<int> g_profile{0};
static std::atomic<int> g_batch_graph{1};
static std::atomic<int> g_force_class{-1};
static std::atomic<int> g_f64_planes{1};
static std::atomic<int> g_crt_wide{-1};  // -1: the tuned class per shape
static std::atomic<int64_t> g_ws_cap{0};

// Environment switches, read once per process: HLB_FORM names the form of calls that pass
// HLB_FORM_AUTO (auto, fp64, int8 or int8_crt); HLB_VALIDATE=1 starts HLB_OPT_VALIDATE on;
// HLB_WS_CAP=<bytes> starts HLB_OPT_WS_CAP at that value (ignored unless a positive integer).
static std::once_flag g_env_once;
static std::atomic<int> g_env_form{HLB_FORM_AUTO};
static std::atomic<int> g_validate{0};
static void read_env() {
    std::call_once(g_env_once, [] {
        if (const char *f = std::getenv("HLB_FORM")) {
            if (!std::strcmp(f, "fp64")) g_env_form.store(HLB_FORM_FP64);
            else if (!std::strcmp(f, "int8")) g_env_form.store(HLB_FORM_INT8);
            else if (!std::strcmp(f, "int8_crt")) g_env_form.store(HLB_FORM_INT8_CRT);
        }
        if (const char *v = std::getenv("HLB_VALIDATE")) g_validate.store(*v && std::strcmp(v, "0") ? 1 : 0);
        if (const char *c = std::getenv("HLB_WS_CAP")) {
            char *end = nullptr;
            const long long v = std::strtoll(c, &end, 10);
            if (end != c && *end == '\0' && v > 0) g_ws_cap.store(v);
        }
    });
}
static int64_t ws_cap() {
    read_env();
    return g_ws_cap.load();
}
int resolve_form(int form) {
    read_env();
    return form == HLB_FORM_AUTO ? g_env_form.load() : form;
}
bool opt_validate() {
    read_env();
    return g_validate.load() != 0;
}

int64_t opt_force_kchunk() { return g_force_kchunk.load(); }
bool opt_batch_graph() { return g_batch_graph.load() != 0; }

struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static std::vector<ProfRec> g_prof;

ProfScope::ProfScope(const char *name, hipStream_t s) : stream_(s) {
    if (!g_profile.load()) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    name_ = name;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) return;
    if (hipEventRecord(a_, s) != hipSuccess) return;
    active_ = true;
}
ProfScope::~ProfScope() {
    if (!active_) return;
    if (hipEventRecord(b_, stream_) != hipSuccess) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back({name_, a_, b_});
}

// ---------------------------------------------------------------------------------------
// Device checks
// ---------------------------------------------------------------------------------------
struct DevInfo {
    int checked = 0;
    bool ok = false;
    int n_xcd = 8;
    int cus = 256;
    bool pool_set = false;
};
static std::mutex g_dev_mu;
static DevInfo g_dev[64];

hlb_status device_ready(int *n_xcd, int *cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return HLB_EDEVICE;
    std::lock_guard<std::mutex> g(g_dev_mu);
    DevInfo &d = g_dev[dev];
    if (!d.checked) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return HLB_EDEVICE;
        d.checked = 1;
        d.ok = std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
        // gfx950 has 32 CUs per XCD; a partitioned device exposes fewer XCDs
        d.n_xcd = std::max(1, p.multiProcessorCount / 32);
        d.cus = std::max(1, p.multiProcessorCount);
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;  // keep freed workspace cached in the pool
            d.pool_set = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr) == hipSuccess;
        }
    }
    if (!d.ok) return HLB_EUNSUP;
    if (n_xcd) *n_xcd = d.n_xcd;
    if (cus) *cus = d.cus;
    return HLB_OK;
}

// ---------------------------------------------------------------------------------------
// Planner (Lemma le:strategy1's exactness condition, per form)
// ---------------------------------------------------------------------------------------

// Largest value representable with D balanced int8 digits: 127 * (256^D - 1) / 255.
static uint64_t i8_capacity(int D) {
    uint64_t c = 0;
    for (int j = 0; j < D; ++j) c = c * 256 + 127;
    return c;
}
static int i8_digits(uint64_t vmax) {
    for (int D = 1; D <= 7; ++D)
        if (vmax <= i8_capacity(D)) return D;
    return 8;
}
int i8_digits_for(uint64_t vmax) { return i8_digits(vmax); }

static int bit_length(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

static int64_t cap_chunk(int64_t chunk, int64_t step) {
    const int64_t f = opt_force_kchunk();
    if (f > 0 && f < chunk) chunk = f;
    chunk = chunk / step * step;
    return chunk;
}

hlb_status plan_i8(int kind, int64_t k, uint64_t qmax, int64_t pmax, Plan *pl) {
    const int dx = i8_digits(qmax - 1);
    const int dp = kind == 0 ? dx : i8_digits((uint64_t)pmax);
    int ip = 0, ix = 0;
    if (dp <= 3 && dx <= 6) ip = 3, ix = 6;
    else if (dp <= 3 && dx == 7) ip = 3, ix = 7;
    else if (dp <= 7 && dx <= 7) ip = 7, ix = 7;
    else return HLB_EBOUND;
    const I8Shape sh = i8_shape(ip, ix, 0);
    if (!sh.dp) return HLB_EBOUND;
    const int pairs = std::min(ip, ix);
    // |c_s| <= pairs * kchunk * 128 * 128 must stay <= 2^31 - 1
    const int64_t limit = ((int64_t)1 << 31) - 1;
    const int64_t chunk = cap_chunk(limit / ((int64_t)pairs * 16384), kBK8);
    if (chunk < kBK8) return HLB_EBOUND;
    pl->form = HLB_FORM_INT8;
    pl->np = ip;
    pl->nx = ix;
    pl->limb_bits = 8;
    pl->pairs = pairs;
    pl->kchunk = chunk;
    pl->bm = sh.bm;
    pl->bn = sh.bn;
    pl->bk = kBK8;
    pl->acc_bound_log2 = std::log2((double)pairs * (double)std::min<int64_t>(k, chunk) * 16384.0);
    return HLB_OK;
}

hlb_status plan_f64(int kind, int64_t k, uint64_t qmax, int64_t pmax, Plan *pl) {
    const double lim = 9007199254740991.0;  // 2^53 - 1
    const int xbits = bit_length(qmax - 1);
    const int64_t kk = std::max<int64_t>(k, 1);
    if (kind == 1) {
        // one signed plaintext limb (k2 = 1), X in NX limbs of w bits:
        // kchunk * pmax * (2^w - 1) < 2^53
        for (int nx = 3; nx <= 4; ++nx) {
            const int w = (xbits + nx - 1) / nx;
            if (w < 1) continue;
            const double per = (double)std::max<int64_t>(pmax, 1) * (double)(((uint64_t)1 << w) - 1);
            const int64_t raw = (int64_t)std::min(lim / per, 4.0e18);
            const int64_t chunk = cap_chunk(raw, kBK64);
            if (chunk >= kBK64 && (chunk >= kk || nx == 4)) {
                pl->form = HLB_FORM_FP64;
                pl->np = 1;
                pl->nx = nx;
                pl->limb_bits = w;
                pl->pairs = 1;
                pl->kchunk = chunk;
                pl->bm = 64;
                pl->bn = 64;
                pl->bk = kBK64;
                pl->acc_bound_log2 = std::log2(per * (double)std::min<int64_t>(kk, chunk));
                return HLB_OK;
            }
        }
    }
    // both operands in L limbs of w bits (P in sign-magnitude limbs):
    // L * kchunk * (2^w - 1)^2 < 2^53
    const int bits = std::max(xbits, kind == 1 ? bit_length((uint64_t)pmax) : xbits);
    for (int L = 3; L <= 4; ++L) {
        const int w = (bits + L - 1) / L;
        const double lm = (double)(((uint64_t)1 << w) - 1);
        const double per = (double)L * lm * lm;
        const int64_t raw = (int64_t)std::min(lim / per, 4.0e18);
        const int64_t chunk = cap_chunk(raw, kBK64);
        if (chunk >= kBK64 && (chunk >= kk || L == 4)) {
            pl->form = HLB_FORM_FP64;
            pl->np = L;
            pl->nx = L;
            pl->limb_bits = w;
            pl->pairs = L;
            pl->kchunk = chunk;
            pl->bm = 64;
            pl->bn = 64;
            pl->bk = kBK64;
            pl->acc_bound_log2 = std::log2(per * (double)std::min<int64_t>(kk, chunk));
            return HLB_OK;
        }
    }
    return HLB_EBOUND;
}

// Truncated b-part plans (Strategy 2 of Section 6.1).
//  INT8: skipping the products P_i X_j with i + j < drop changes the integer result by
//        D = sum_{i+j<drop} (P_i X_j) 256^(i+j) with |P_i X_j| <= k * 2^14 per entry, so
//        |D| <= k 2^14 sum_{s<drop} pairs(s) 256^s.  Only without a K fold (k <= kchunk).
//  FP64: one product of the rounded operands; |P| <= pmax and |centred X| <= q/2, so each of
//        the k terms is at most pmax q/2 and any summation order with faithfully rounded
//        operations is within (k + 2) 2^-52 sum |terms| of the exact value.  The result is
//        exact when every partial sum stays below 2^53.  The epilogue needs |acc| < q 2^51,
//        which k * pmax <= 2^51 guarantees.
hlb_status plan_trunc_b(int64_t k, uint64_t qmin, uint64_t qmax, int64_t pmax, double err_log2, int form, Plan *pl) {
    hlb_status st = plan(1, k, qmax, pmax, form, pl);
    if (st != HLB_OK) return st;
    const double half_qmin = std::log2((double)qmin) - 1.0;
    const double kk = (double)std::max<int64_t>(k, 1);
    if (pl->form == HLB_FORM_INT8_CRT) return HLB_OK;  // no truncated variant: the exact plan
    if (pl->form == HLB_FORM_INT8) {
        if (pl->np != 3 || k > pl->kchunk) return HLB_OK;
        for (int drop = 3; drop >= 1; --drop) {
            double sum = 0.0;
            for (int s = 0; s < drop; ++s) {
                int pairs = 0;
                for (int i = 0; i < pl->np; ++i)
                    if (s - i >= 0 && s - i < pl->nx) ++pairs;
                sum += pairs * std::ldexp(1.0, 8 * s);
            }
            const double bound = std::log2(kk * 16384.0 * sum);
            if (bound <= err_log2 && bound < half_qmin) {
                pl->drop = drop;
                pl->err_bound_log2 = bound;
                return HLB_OK;
            }
        }
        return HLB_OK;
    }
    // FP64
    const double terms = kk * (double)std::max<int64_t>(pmax, 1) * (double)(qmax / 2);
    if (kk * (double)std::max<int64_t>(pmax, 1) > std::ldexp(1.0, 51)) return HLB_OK;
    const double bound = terms < std::ldexp(1.0, 53) ? -__builtin_inf() : std::log2((kk + 2.0) * std::ldexp(terms, -52));
    if (bound <= err_log2 && bound < half_qmin) {
        pl->trunc = true;
        pl->np = 1;
        pl->nx = 1;
        pl->limb_bits = 0;
        pl->pairs = 1;
        pl->kchunk = INT64_MAX / 2;
        pl->acc_bound_log2 = std::log2(std::max(terms, 1.0));
        pl->err_bound_log2 = bound;
    }
    return HLB_OK;
}

// Multimodular plan (Strategy 3): the centred product satisfies |V| <= k * a * b with
// a = p_absmax (plaintext) or floor(q/2) (residues) and b = floor(q/2); the first D moduli
// must multiply to at least 4 |V| (so that |V| / M <= 1/4), and |c| <= k 2^14 < 2^31.
hlb_status plan_crt(int kind, int64_t k, uint64_t qmax, int64_t pmax, Plan *pl) {
    if (k > 131071) return HLB_EBOUND;
    const double half_q = (double)(qmax / 2 > 0 ? qmax / 2 : 1);
    const double a = kind == 1 ? (double)std::max<int64_t>(pmax, 1) : half_q;
    const double need = std::log2((double)std::max<int64_t>(k, 1)) + std::log2(a) + std::log2(half_q) + 2.0;
    double have = 0.0;
    int D = 0;
    while (D < kCrtMaxModuli && have < need) have += std::log2((double)kCrtModuli[D++]);
    if (have < need) return HLB_EBOUND;
    D = crt_round_d(D);
    if (D == 0) return HLB_EBOUND;
    pl->form = HLB_FORM_INT8_CRT;
    pl->np = D;
    pl->nx = D;
    pl->limb_bits = 8;
    pl->pairs = 1;
    pl->kchunk = std::max<int64_t>(k, kBK8);
    pl->bm = 256;
    pl->bn = 128;
    pl->bk = kBK8;
    pl->acc_bound_log2 = std::log2((double)std::max<int64_t>(k, 1) * 16384.0);
    return HLB_OK;
}

hlb_status plan(int kind, int64_t k, uint64_t qmax, int64_t pmax, int form, Plan *pl) {
    pl->kind = kind;
    if (form == HLB_FORM_INT8) return plan_i8(kind, k, qmax, pmax, pl);
    if (form == HLB_FORM_FP64) return plan_f64(kind, k, qmax, pmax, pl);
    if (form == HLB_FORM_INT8_CRT) return plan_crt(kind, k, qmax, pmax, pl);
    if (form == HLB_FORM_AUTO) {
        // the multimodular form when its D int8 products clearly undercut the digit pairs
        // (both measured at d = 8192: 11 moduli at 50-51 % of the int8 peak beat 21 digit
        // pairs at 49 %, 1.8x faster per CP-MM); the digit form otherwise, FP64 where no int8
        // plan exists
        Plan digit, crt;
        digit.kind = crt.kind = kind;
        const bool has_digit = plan_i8(kind, k, qmax, pmax, &digit) == HLB_OK;
        const bool has_crt = plan_crt(kind, k, qmax, pmax, &crt) == HLB_OK;
        if (has_crt && (!has_digit || 4 * crt.np < 3 * digit.np * digit.nx)) {
            *pl = crt;
            return HLB_OK;
        }
        if (has_digit) {
            *pl = digit;
            return HLB_OK;
        }
        return plan_f64(kind, k, qmax, pmax, pl);
    }
    return HLB_EINVAL;
}

// ---------------------------------------------------------------------------------------
// Tile-class tuning table: (x digits, log2 m, log2 n, log2 k) -> class.
// ---------------------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<uint32_t, int> g_tune;
static bool g_tune_env_loaded = false;

static int floor_log2(int64_t v) { return v <= 1 ? 0 : 63 - __builtin_clzll((unsigned long long)v); }
static uint32_t tune_key(int dx, int lm, int ln, int lk) {
    return ((uint32_t)(dx & 0xff) << 24) | ((uint32_t)(lm & 0x3f) << 12) | ((uint32_t)(ln & 0x3f) << 6) |
           (uint32_t)(lk & 0x3f);
}
// Multimodular entries share the table under the first key field 0x80 | moduli count.
static uint32_t tune_key_crt(int moduli, int lm, int ln, int lk) { return tune_key(0x80 | moduli, lm, ln, lk); }
static bool tune_fields_ok(int lm, int ln, int lk) {
    return lm >= 0 && lm <= 63 && ln >= 0 && ln <= 63 && lk >= 0 && lk <= 63;
}
static hlb_status tune_load_locked(const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return HLB_EINVAL;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        int dx, lm, ln, lk, c;
        if (std::sscanf(line, " crt %d %d %d %d %d", &dx, &lm, &ln, &lk, &c) == 5) {
            if (dx >= 1 && dx <= kCrtMaxModuli && tune_fields_ok(lm, ln, lk) && c >= 0 && c <= 2)
                g_tune[tune_key_crt(dx, lm, ln, lk)] = c;
        } else if (std::sscanf(line, "%d %d %d %d %d", &dx, &lm, &ln, &lk, &c) == 5 && dx >= 1 && dx <= 8 &&
                   tune_fields_ok(lm, ln, lk) && (c == 0 || c == 1)) {
            g_tune[tune_key(dx, lm, ln, lk)] = c;
        }
    }
    std::fclose(f);
    return HLB_OK;
}
static int tune_lookup(int dx, int64_t m, int64_t n, int64_t k) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!g_tune_env_loaded) {
        g_tune_env_loaded = true;
        const char *env = std::getenv("HLB_TUNE_CACHE");
        if (env && *env) (void)tune_load_locked(env);
    }
    auto it = g_tune.find(tune_key(dx, floor_log2(m), floor_log2(n), floor_log2(k)));
    return it == g_tune.end() ? -1 : it->second;
}

// The multimodular GEMM's tile class for a product of D moduli, m rows, n columns (of one
// output matrix) and depth k: the forced class (HLB_OPT_CRT_WIDE), else the tuned one, else
// 256 x 384 (2), the widest, which holds the most MFMAs per wave and stage.
int crt_tile_class(int D, int64_t m, int64_t n, int64_t k) {
    const int forced = g_crt_wide.load();
    if (forced >= 0) return forced;
    const int c = tune_lookup(0x80 | D, std::max<int64_t>(m, 1), std::max<int64_t>(n, 1), std::max<int64_t>(k, 1));
    return c >= 0 ? c : 2;
}

// AUTO picks the multimodular form by depth alone; its 256 x 384 output tiles would be mostly
// padding on a small product, so there the digit plan is taken instead.
static void auto_for_shape(Plan *pl, int form, int64_t m, int64_t n, int64_t k, uint64_t qmax, int64_t pmax) {
    if (form != HLB_FORM_AUTO || pl->form != HLB_FORM_INT8_CRT || (m >= 256 && n >= 256)) return;
    Plan digit;
    digit.kind = pl->kind;
    if (plan_i8(pl->kind, k, qmax, pmax, &digit) == HLB_OK) *pl = digit;
}

void choose_class(Plan *pl, int64_t m, int64_t n, int64_t k) {
    if (pl->form != HLB_FORM_INT8 || pl->np != 3) return;
    int cls = g_force_class.load();
    if (cls < 0) cls = tune_lookup(pl->nx, m, n, k);
    if (cls < 0) {
        // padding waste: rows padded to the tile height, columns to the tile width
        const I8Shape a = i8_shape(pl->np, pl->nx, 0), b = i8_shape(pl->np, pl->nx, 1);
        auto padded = [&](const I8Shape &sh) {
            return (double)((m + sh.bm - 1) / sh.bm * sh.bm) * (double)((n + sh.bn - 1) / sh.bn * sh.bn);
        };
        cls = padded(b) < padded(a) ? 1 : 0;
    }
    const I8Shape sh = i8_shape(pl->np, pl->nx, cls);
    if (!sh.dp) return;
    pl->cls = cls;
    pl->bm = sh.bm;
    pl->bn = sh.bn;
}

void fill_seg(Seg &s, uint64_t q, int limb_bits) {
    s.q = q;
    s.qinv = 1.0 / (double)q;
    const unsigned __int128 w = ((unsigned __int128)1 << limb_bits) % q;
    s.wmod = (uint64_t)w;
    s.wshoup = (uint64_t)((w << 64) / q);
}

hlb_status check_modulus(uint64_t q) { return (q >= 2 && q < kMaxModulus) ? HLB_OK : HLB_EINVAL; }

// ---------------------------------------------------------------------------------------
// Workspace: stream-ordered allocations from the device's default pool (kept cached).
// ---------------------------------------------------------------------------------------
// Sizes are rounded up to one of four steps per power of two (at most 25 % more), so that
// calls of varying shapes ask the pool for few distinct sizes and reuse its cached blocks
// instead of mapping new memory on every call.
static size_t ws_bucket(size_t bytes) {
    if (bytes <= ((size_t)1 << 16)) return (size_t)1 << 16;
    int e = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t step = (size_t)1 << (e - 2);
    return (bytes + step - 1) / step * step;
}

hlb_status ws_alloc(void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) return HLB_OK;
    const int64_t cap = ws_cap();
    if (cap > 0 && ws_bucket(bytes) > (size_t)cap) return HLB_ENOMEM;
    if (hipMallocAsync(p, ws_bucket(bytes), s) != hipSuccess) {
        (void)hipGetLastError();
        return HLB_ENOMEM;
    }
    return HLB_OK;
}
void ws_free(void *p, hipStream_t s) {
    if (p) (void)hipFreeAsync(p, s);
}

// Per-stream blocks.  A pool allocation per call was measured to degrade: after a few hundred
// calls alternating shapes and forms, hipMallocAsync averaged 1.3 ms and reached seconds.
// Each slot records an event on its stream when a call's lease ends; the next call that takes
// the block waits for it on its own stream first.  Calls on one stream are ordered anyway, but
// a destroyed stream's handle may be handed to a new stream, whose work would otherwise not
// be ordered after the old stream's use of the block.  A device keeps at most kMaxSlotBlocks
// blocks: taking one beyond that frees the least recently used idle block (after its event).
struct WsSlot {
    std::mutex mu;  // held by the lease of the call using the block
    void *p = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;  // recorded on the stream at the end of each lease
    uint64_t last_use = 0;
    int dev = 0;
};
static std::mutex g_slots_mu;
static std::map<std::pair<int, hipStream_t>, WsSlot *> g_slots;
static uint64_t g_slot_tick = 0;  // guarded by g_slots_mu
constexpr int kMaxSlotBlocks = 4;

// Frees idle blocks of device `dev` (least recently used first) until at most keep - 1 other
// blocks remain besides `self`; a block still in use by another thread is skipped.
static void ws_evict_lru(int dev, const WsSlot *self, hipStream_t s, int keep) {
    std::lock_guard<std::mutex> g(g_slots_mu);
    std::vector<WsSlot *> held;
    for (auto &kv : g_slots)
        if (kv.second != self && kv.second->dev == dev && kv.second->p) held.push_back(kv.second);
    if ((int)held.size() < keep) return;
    std::sort(held.begin(), held.end(), [](const WsSlot *a, const WsSlot *b) { return a->last_use < b->last_use; });
    for (size_t i = 0; i + (size_t)keep <= held.size(); ++i) {
        WsSlot *v = held[i];
        if (!v->mu.try_lock()) continue;
        if (v->done) (void)hipEventSynchronize(v->done);
        if (v->p) (void)hipFreeAsync(v->p, s);
        v->p = nullptr;
        v->bytes = 0;
        v->mu.unlock();
    }
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// The calling thread's scratch span while a ScratchScope is alive (the no-allocation entry
// point): the lease then carves its buffers from the span and allocates nothing.
static thread_local const ScratchScope *t_scratch = nullptr;

ScratchScope::ScratchScope(void *base, size_t bytes) : base_(base), bytes_(bytes), prev_(t_scratch) {
    t_scratch = this;
}
ScratchScope::~ScratchScope() { t_scratch = prev_; }

hlb_status WsLease::take(hipStream_t s, const size_t *bytes, void **ptrs, int n) {
    const ScratchScope *scr = t_scratch;
    const int64_t cap = scr ? 0 : ws_cap();
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        ptrs[i] = nullptr;
        if (bytes[i] == 0) continue;
        if (cap > 0 && ws_bucket(bytes[i]) > (size_t)cap) return HLB_ENOMEM;
        total += align256(bytes[i]);
    }
    if (total == 0) return HLB_OK;
    s_ = s;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    char *base = nullptr;
    if (scr) {
        if (total > scr->bytes()) return HLB_ESCRATCH;
        base = (char *)scr->base();
    } else if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        if (hipMallocAsync(&own_, total, s) != hipSuccess) {
            (void)hipGetLastError();
            own_ = nullptr;
            return HLB_ENOMEM;
        }
        base = (char *)own_;
    } else {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return HLB_EDEVICE;
        {
            std::lock_guard<std::mutex> g(g_slots_mu);
            WsSlot *&sl = g_slots[{dev, s}];
            if (!sl) {
                sl = new WsSlot;
                sl->dev = dev;
            }
            slot_ = sl;
            slot_->last_use = ++g_slot_tick;
        }
        slot_->mu.lock();
        // work enqueued on this stream handle before (possibly by a stream since destroyed)
        if (slot_->done && hipStreamWaitEvent(s, slot_->done, 0) != hipSuccess) {
            (void)hipGetLastError();
            return HLB_EDEVICE;  // the destructor unlocks
        }
        if (!slot_->p) ws_evict_lru(dev, slot_, s, kMaxSlotBlocks);
        if (slot_->bytes < total) {
            // the old block's last users precede this call in stream order
            if (slot_->p) (void)hipFreeAsync(slot_->p, s);
            slot_->p = nullptr;
            slot_->bytes = 0;
            const size_t want = ws_bucket(total);
            if (hipMallocAsync(&slot_->p, want, s) != hipSuccess) {
                (void)hipGetLastError();
                slot_->p = nullptr;
                return HLB_ENOMEM;  // the destructor unlocks
            }
            slot_->bytes = want;
        }
        base = (char *)slot_->p;
    }
    for (int i = 0; i < n; ++i) {
        if (bytes[i] == 0) continue;
        ptrs[i] = base;
        base += align256(bytes[i]);
    }
    return HLB_OK;
}

WsLease::~WsLease() {
    if (own_) (void)hipFreeAsync(own_, s_);
    if (slot_) {
        if (!slot_->done && hipEventCreateWithFlags(&slot_->done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            slot_->done = nullptr;
        }
        if (slot_->done && hipEventRecord(slot_->done, s_) != hipSuccess) (void)hipGetLastError();
        slot_->mu.unlock();
    }
}

// Frees every stream's block (the device work that used them must have completed).
void ws_release_all() {
    std::lock_guard<std::mutex> g(g_slots_mu);
    for (auto &kv : g_slots) {
        std::lock_guard<std::mutex> h(kv.second->mu);
        if (kv.second->p) (void)hipFreeAsync(kv.second->p, nullptr);
        kv.second->p = nullptr;
        kv.second->bytes = 0;
    }
    (void)hipDeviceSynchronize();
}

// ---------------------------------------------------------------------------------------
// One GEMM launch over up to kMaxSegs output segments sharing the left operand.
// ---------------------------------------------------------------------------------------
// Multimodular form of run_products: residue splits of every right operand and of each left
// operand, one INT8 GEMM launch per left operand and group of up to kMaxSegs right operands
// (all D moduli in one grid), then one recombination launch per output matrix.
static hlb_status run_products_crt(const Plan &pl, const std::vector<LeftSpec> &lefts,
                                   const std::vector<RightSpec> &rights, int64_t k, int n_xcd, hipStream_t s) {
    const int D = pl.np;
    int64_t mmax0 = 0, nmax0 = 0;
    for (const LeftSpec &L : lefts) mmax0 = std::max(mmax0, L.m);
    for (const RightSpec &R : rights) nmax0 = std::max(nmax0, R.n);
    const int wide = crt_tile_class(D, mmax0, nmax0, k);
    int cus = 256;
    (void)device_ready(nullptr, &cus);
    const int64_t bn = crt_tile_cols(wide), xsub = bn / 128;
    // The persistent launch of the 256 x 384 tiles takes even K-block counts only: an odd count
    // of at least kCrtPadOddKB gets one more block, all zeros (the splits write zeros past k),
    // which costs less than the per-tile launch it avoids (measured: the persistent launch saves
    // 2-3 us per tile, 2-10 % of a tile at these depths; the block adds 1/KB of the work).
    constexpr int64_t kCrtPadOddKB = 15;
    int64_t kblocks = (k + kBK8 - 1) / kBK8;
    if (wide == 2 && kblocks % 2 == 1 && kblocks >= kCrtPadOddKB) ++kblocks;
    const int64_t sub = (int64_t)D * 128 * kBK8;  // bytes of one 128-wide tile and k block
    int64_t mmax = 0;
    for (const LeftSpec &L : lefts) mmax = std::max(mmax, L.m);
    const int64_t t128_m = ((mmax + 255) / 256) * 2;  // 128-row tiles, even: GEMM tiles are 256 rows
    // per right operand: its 128-column split tiles.  The right operands of one GEMM launch lie
    // side by side, and its GEMM tiles (xsub split tiles wide) may straddle two of them; the
    // last may reach up to xsub - 1 split tiles past the end, so the workspace has them too.
    std::vector<int64_t> t128_n(rights.size());
    int64_t tn_total = 0, ybytes = 0;
    for (size_t i = 0; i < rights.size(); ++i) {
        t128_n[i] = (rights[i].n + 127) / 128;
        tn_total += t128_n[i];
        // product planes cover whole 256-row and 128-column tiles (layout of CrtSeg)
        ybytes += (int64_t)D * (t128_m / 2 * 256) * (t128_n[i] * 128);
    }
    if (kblocks > INT32_MAX / 2 || t128_m * kblocks > INT32_MAX / 2 || (tn_total + xsub) * kblocks > INT32_MAX / 2 ||
        (int64_t)D * (t128_m / 2) * (tn_total + xsub) > INT32_MAX / 2)
        return HLB_EINVAL;

    // constants: M = prod p_i, inv_i = (M / p_i)^{-1} mod p_i
    unsigned __int128 M = 1;
    for (int i = 0; i < D; ++i) M *= (unsigned)kCrtModuli[i];
    CrtScale inv;
    std::memset(&inv, 0, sizeof(inv));
    for (int i = 0; i < D; ++i) {
        const int p = kCrtModuli[i];
        const int mi = (int)((M / (unsigned)p) % (unsigned)p);
        for (int v = 1; v < p; ++v)
            if ((mi * v) % p == 1) {
                inv.s[i] = v;
                break;
            }
    }

    void *wsP = nullptr, *wsX = nullptr, *wsY = nullptr, *wsC = nullptr;
    WsLease lease;
    {
        // planes of the left and right operands, product planes, tile-queue counters
        const size_t sizes[4] = {(size_t)(t128_m * kblocks * sub), (size_t)((tn_total + xsub - 1) * kblocks * sub),
                                 (size_t)ybytes, kMaxChunks * sizeof(unsigned int)};
        void *ptrs[4];
        const hlb_status st = lease.take(s, sizes, ptrs, 4);
        if (st != HLB_OK) return st;
        wsP = ptrs[0];
        wsX = ptrs[1];
        wsY = ptrs[2];
        wsC = ptrs[3];
    }
    // offsets of each right operand's split tiles (128 wide) and product planes
    std::vector<int64_t> x_tile0(rights.size()), y_off(rights.size());
    {
        int64_t t0 = 0, y0 = 0;
        for (size_t i = 0; i < rights.size(); ++i) {
            x_tile0[i] = t0;
            y_off[i] = y0;
            t0 += t128_n[i];
            y0 += (int64_t)D * (t128_m / 2 * 256) * (t128_n[i] * 128);
        }
    }
    // a left operand holding residues is centred modulo the (shared) modulus of the products
    const uint64_t left_qc = pl.kind == 0 ? rights[0].q : 0;
    // Splits go out in launches of up to kCrtTabSplit operands (the job table travels in the
    // kernel arguments): every right operand, and the left operand too when there is only one.
    CrtSplitTable stab;
    int64_t swgs = 0;
    auto split_reset = [&]() {
        std::memset(&stab, 0, sizeof(stab));
        for (int i = 0; i < kCrtTabSplit; ++i) stab.start[i] = INT32_MAX;
        swgs = 0;
    };
    split_reset();
    auto split_flush = [&](hipStream_t st) -> bool {
        if (stab.njobs == 0) return true;
        ProfScope ps("crt_split", st);
        const bool ok = launch_crt_split_tab(D, stab, swgs, inv, st) == hipSuccess;
        split_reset();
        return ok;
    };
    auto split_add = [&](const CrtSplitJob &j, int64_t wgs, hipStream_t st) -> bool {
        if ((stab.njobs == kCrtTabSplit || swgs + wgs > INT32_MAX / 2) && !split_flush(st)) return false;
        if (wgs > INT32_MAX / 2) return false;
        stab.start[stab.njobs] = (int32_t)swgs;
        CrtSplitJob &e = stab.job[stab.njobs++];
        e = j;
        e.wg_start = swgs;
        swgs += wgs;
        return true;
    };
    auto split_x = [&](size_t i, hipStream_t st) -> bool {
        CrtSplitJob j;
        std::memset(&j, 0, sizeof(j));
        j.src = rights[i].X;
        j.ld = rights[i].ldx;
        j.extent = rights[i].n;
        j.k = k;
        j.qc = rights[i].q;
        j.kblocks = (int32_t)kblocks;
        j.rows_side = 0;
        j.out = (int8_t *)wsX + x_tile0[i] * kblocks * sub;
        return split_add(j, t128_n[i] * kblocks, st);
    };
    auto split_p = [&](const LeftSpec &L, hipStream_t st) -> bool {
        const int64_t lt = ((L.m + 255) / 256) * 2;
        CrtSplitJob j;
        std::memset(&j, 0, sizeof(j));
        j.src = L.P;
        j.ld = L.ldp;
        j.extent = L.m;
        j.k = k;
        j.qc = left_qc;
        j.kblocks = (int32_t)kblocks;
        j.rows_side = 1;
        j.out = (int8_t *)wsP;
        return split_add(j, lt * kblocks, st);
    };
    // product planes of right operand i for left operand L
    auto segment = [&](const LeftSpec &L, size_t i) {
        CrtSeg sg;
        std::memset(&sg, 0, sizeof(sg));
        const int64_t lt = ((L.m + 255) / 256) * 2;
        sg.Y = (uint8_t *)wsY + y_off[i];
        sg.n = rights[i].n;
        sg.nbc = t128_n[i] * 4;
        sg.plane = (lt / 2 * 256) * (t128_n[i] * 128);
        sg.tiles = (int32_t)t128_n[i];
        return sg;
    };
    // one GEMM launch for right operands [first, last), all D moduli
    auto gemm = [&](const LeftSpec &L, size_t first, size_t last, hipStream_t st) -> bool {
        CrtGemmArgs a;
        std::memset(&a, 0, sizeof(a));
        a.Pd = (const int8_t *)wsP;
        a.Xd = (const int8_t *)wsX + x_tile0[first] * kblocks * sub;
        a.m = L.m;
        a.kblocks = (int)kblocks;
        a.D = D;
        a.tiles_m = (int)((L.m + 255) / 256);
        // 8 row tiles per raster group: the 32 tiles an XCD runs at once then share 8 left and
        // 4 right operand panels (measured at d = 8192: 2, 4, 8, 16 -> 34.6, 32.8, 32.0, 33.2 ms)
        a.group_m = 8;
        a.n_xcd = n_xcd;
        a.counters = (unsigned int *)wsC;
        int32_t tb = 0;
        for (size_t i = first; i < last; ++i) {
            CrtSeg &sg = a.seg[a.nseg++];
            sg = segment(L, i);
            sg.tile_begin = tb;
            tb += (int32_t)t128_n[i];
        }
        a.tiles_n = (int32_t)((tb + xsub - 1) / xsub);
        if (tb == 0) return true;
        ProfScope ps("crt_gemm", st);
        return launch_crt_gemm(wide, a, cus, st) == hipSuccess;
    };
    // Recombinations go out in launches of up to kCrtTabCombine output matrices.
    CrtCombineTable ctab;
    int64_t cwgs = 0;
    auto combine_reset = [&]() {
        std::memset(&ctab, 0, sizeof(ctab));
        for (int i = 0; i < kCrtTabCombine; ++i) ctab.start[i] = INT32_MAX;
        cwgs = 0;
    };
    combine_reset();
    auto combine_flush = [&](hipStream_t st) -> bool {
        if (ctab.njobs == 0) return true;
        ProfScope ps("crt_combine", st);
        const bool ok = launch_crt_combine_tab(ctab, cwgs, st) == hipSuccess;
        combine_reset();
        return ok;
    };
    auto combine = [&](const LeftSpec &L, size_t i, hipStream_t st) -> bool {
        if (rights[i].n == 0) return true;
        const CrtSeg sg = segment(L, i);
        const int64_t wgs = crt_combine_wgs(L.m, sg.n);
        if ((ctab.njobs == kCrtTabCombine || cwgs + wgs > INT32_MAX / 2) && !combine_flush(st)) return false;
        if (wgs > INT32_MAX / 2) return false;
        ctab.start[ctab.njobs] = (int32_t)cwgs;
        CrtCombineJob &j = ctab.job[ctab.njobs++];
        std::memset(&j, 0, sizeof(j));
        j.wg_start = cwgs;
        cwgs += wgs;
        CrtCombineArgs &c = j.a;
        c.Y = sg.Y;
        c.C = L.C[i];
        c.m = L.m;
        c.n = sg.n;
        c.nbc = sg.nbc;
        c.plane = sg.plane;
        c.ldc = L.ldc[i];
        c.q = rights[i].q;
        c.barrett = (uint64_t)((~(unsigned __int128)0 >> 64) / c.q);
        c.Mq = (uint64_t)(M % c.q);
        c.D = D;
        for (int jj = 0; jj < D; ++jj) c.w[jj] = (uint64_t)((M / (unsigned)kCrtModuli[jj]) % c.q);
        return true;
    };

    // one left operand: its split joins the right operands' (the planes of P are shared by
    // every GEMM launch); several: each is split before its own GEMMs, into the same planes
    const bool one_left = lefts.size() == 1;
    if (one_left && lefts[0].m > 0 && !split_p(lefts[0], s)) return HLB_EDEVICE;
    for (size_t i = 0; i < rights.size(); ++i)
        if (!split_x(i, s)) return HLB_EDEVICE;
    if (!split_flush(s)) return HLB_EDEVICE;
    for (const LeftSpec &L : lefts) {
        if (L.m == 0) continue;
        if (!one_left && (!split_p(L, s) || !split_flush(s))) return HLB_EDEVICE;
        for (size_t first = 0; first < rights.size(); first += kMaxSegs) {
            const size_t last = std::min(rights.size(), first + kMaxSegs);
            if (!gemm(L, first, last, s)) return HLB_EDEVICE;
            for (size_t i = first; i < last; ++i)
                if (!combine(L, i, s)) return HLB_EDEVICE;
            if (!combine_flush(s)) return HLB_EDEVICE;
        }
    }
    return HLB_OK;
}

// Runs C[l][r] = L_l * X_r mod q_r for every left operand L_l and right operand X_r.  Each
// right operand is split once and shared by all left operands; each left operand is split
// once and shared by all right operands; then one GEMM launch per left operand covers up to
// kMaxSegs right operands (more are chunked).
hlb_status run_products(const Plan &pl, const std::vector<LeftSpec> &lefts, const std::vector<RightSpec> &rights,
                        int64_t k, int n_xcd, hipStream_t s) {
    if (lefts.empty() || rights.empty()) return HLB_OK;
    int64_t mmax = 0;
    for (const LeftSpec &L : lefts) mmax = std::max(mmax, L.m);
    if (mmax == 0) return HLB_OK;
    if (k == 0) {
        for (const LeftSpec &L : lefts)
            for (size_t r = 0; r < rights.size(); ++r)
                if (launch_zero(L.C[r], L.m, rights[r].n, L.ldc[r], s) != hipSuccess) return HLB_EDEVICE;
        return HLB_OK;
    }
    if (pl.form == HLB_FORM_INT8_CRT) return run_products_crt(pl, lefts, rights, k, n_xcd, s);
    const int64_t tiles_mmax = (mmax + pl.bm - 1) / pl.bm;
    const int64_t kblocks = (k + pl.bk - 1) / pl.bk;
    const int64_t kfold = std::max<int64_t>(1, pl.kchunk / pl.bk);
    std::vector<int64_t> seg_tiles(rights.size());
    int64_t tiles_total = 0;
    for (size_t i = 0; i < rights.size(); ++i) {
        seg_tiles[i] = (rights[i].n + pl.bn - 1) / pl.bn;
        tiles_total += seg_tiles[i];
    }
    // grid sizes and in-kernel tile indices are 32-bit
    if (kblocks > INT32_MAX / 2 || tiles_total > INT32_MAX / 2 || tiles_mmax * tiles_total > INT32_MAX / 2)
        return HLB_EINVAL;

    void *wsP = nullptr, *wsX = nullptr;
    // FP64 plans with one plaintext limb run on prepared double planes (unless switched off)
    bool planes = pl.form == HLB_FORM_FP64 && pl.np == 1 && g_f64_planes.load() != 0 &&
                  (pl.trunc ? pl.nx == 1 : (pl.nx == 3 || pl.nx == 4));
    // the plane tiles address their K panels with 32-bit byte offsets: a deeper K stays on
    // the register-staged kernel
    if (planes && kblocks * f64_plane_bytes_x(pl.nx, 1, 1) > (int64_t)UINT32_MAX) planes = false;
    int64_t p_tile = (int64_t)pl.np * pl.bm * kBK8, x_tile = (int64_t)pl.nx * pl.bn * kBK8;
    if (planes) {
        p_tile = f64_plane_bytes_p(1, 1);
        x_tile = f64_plane_bytes_x(pl.nx, 1, 1);
    }
    // the INT8 tiles address their digit panels with 32-bit byte offsets
    if (pl.form == HLB_FORM_INT8 && kblocks * std::max(p_tile, x_tile) > (int64_t)UINT32_MAX) return HLB_EINVAL;
    WsLease lease;
    if (pl.form == HLB_FORM_INT8 || planes) {
        const size_t sizes[2] = {(size_t)(tiles_mmax * kblocks * p_tile), (size_t)(tiles_total * kblocks * x_tile)};
        void *ptrs[2];
        const hlb_status st = lease.take(s, sizes, ptrs, 2);
        if (st != HLB_OK) return st;
        wsP = ptrs[0];
        wsX = ptrs[1];
        int64_t t0 = 0;
        for (size_t i = 0; i < rights.size(); ++i) {
            ProfScope ps(planes ? "prep_x" : "split_x", s);
            int8_t *dst = (int8_t *)wsX + t0 * kblocks * x_tile;
            const hipError_t e =
                planes ? launch_prep_x_planes(pl.nx, pl.trunc, rights[i].X, rights[i].ldx, k, rights[i].n,
                                              (int)seg_tiles[i], (int)kblocks, pl.limb_bits, rights[i].q,
                                              (double *)dst, s)
                       : launch_split_cols_i8(pl.nx, pl.bn, rights[i].X, rights[i].ldx, k, rights[i].n,
                                              (int)seg_tiles[i], (int)kblocks, dst, s);
            if (e != hipSuccess) {
                return HLB_EDEVICE;
            }
            t0 += seg_tiles[i];
        }
    }

    for (const LeftSpec &L : lefts) {
        if (L.m == 0) continue;
        const int64_t tiles_m = (L.m + pl.bm - 1) / pl.bm;
        if (pl.form == HLB_FORM_INT8 || planes) {
            // stream order: this split runs after the previous left operand's GEMM has read wsP
            ProfScope ps(planes ? "prep_p" : "split_p", s);
            const hipError_t e =
                planes ? launch_prep_p_planes(L.P, L.ldp, L.m, k, (int)tiles_m, (int)kblocks, (double *)wsP, s)
                       : launch_split_rows_i8(pl.np, pl.bm, L.P, L.ldp, L.m, k, (int)tiles_m, (int)kblocks,
                                              (int8_t *)wsP, s);
            if (e != hipSuccess) {
                return HLB_EDEVICE;
            }
        }
        int64_t tile_base = 0;
        for (size_t first = 0; first < rights.size(); first += kMaxSegs) {
            const size_t last = std::min(rights.size(), first + kMaxSegs);
            GemmArgs a;
            std::memset(&a, 0, sizeof(a));
            a.Pd = (const int8_t *)wsP;
            a.Xd = wsX ? (const int8_t *)wsX + tile_base * kblocks * x_tile : nullptr;
            a.P = L.P;
            a.ldp = L.ldp;
            a.m = L.m;
            a.k = k;
            a.kblocks = (int)kblocks;
            a.kfold = kfold >= kblocks ? (int)kblocks + 1 : (int)kfold;  // >= kblocks: no fold
            a.tiles_m = (int)tiles_m;
            // 4 row tiles per raster group.  For the digit GEMM, 16 was 1.5 % faster at d = 8192
            // but read 1.3x the HBM bytes there and 1.4x at d = 16384, where it was slower.
            a.group_m = 4;
            a.n_xcd = n_xcd;
            a.limb_bits = pl.limb_bits;
            int32_t tb = 0;
            for (size_t i = first; i < last; ++i) {
                Seg &sg = a.seg[a.nseg++];
                sg.C = L.C[i];
                sg.X = rights[i].X;
                sg.ldc = L.ldc[i];
                sg.ldx = rights[i].ldx;
                sg.n = rights[i].n;
                fill_seg(sg, rights[i].q, pl.limb_bits);
                sg.tile_begin = tb;
                sg.tiles = (int32_t)seg_tiles[i];
                tb += sg.tiles;
            }
            a.tiles_n = tb;
            tile_base += tb;
            if (tb == 0) continue;
            hipError_t e;
            if (pl.form == HLB_FORM_INT8 && pl.drop > 0) {
                ProfScope ps("gemm_i8_trunc", s);
                e = launch_gemm_i8_trunc(pl.np, pl.nx, pl.cls, pl.drop, a, s);
            } else if (pl.form == HLB_FORM_INT8) {
                ProfScope ps("gemm_i8", s);
                e = launch_gemm_i8(pl.np, pl.nx, pl.cls, a, s);
            } else if (planes) {
                ProfScope ps(pl.trunc ? "gemm_f64_trunc" : "gemm_f64", s);
                e = launch_gemm_f64_planes(pl.nx, pl.trunc, a, s);
            } else if (pl.trunc) {
                ProfScope ps("gemm_f64_trunc", s);
                e = launch_gemm_f64_trunc(a, s);
            } else {
                ProfScope ps("gemm_f64", s);
                e = launch_gemm_f64(pl.np, pl.nx, a, s);
            }
            if (e != hipSuccess) {
                return HLB_EDEVICE;
            }
        }
    }
    return HLB_OK;
}

// True when `s` is being captured into a graph (or its capture state cannot be read).
bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Synchronous reduction with a host result: refused (before anything is enqueued) on a stream
// under capture, where neither the copy to the host nor the synchronization may happen.
hlb_status measure_absmax(const int64_t *P, int64_t m, int64_t k, int64_t ld, int64_t *out, hipStream_t s) {
    if (stream_capturing(s)) return HLB_EINVAL;
    unsigned long long *d = nullptr;
    if (hipMallocAsync((void **)&d, sizeof(*d), s) != hipSuccess) {
        (void)hipGetLastError();
        return HLB_ENOMEM;
    }
    hlb_status st = HLB_OK;
    if (launch_zero((uint64_t *)d, 1, 1, 1, s) != hipSuccess) st = HLB_EDEVICE;
    if (st == HLB_OK && m > 0 && k > 0 && launch_absmax(P, m, k, ld, d, s) != hipSuccess) st = HLB_EDEVICE;
    unsigned long long h = 0;
    if (st == HLB_OK && hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) st = HLB_EDEVICE;
    (void)hipFreeAsync(d, s);
    if (hipStreamSynchronize(s) != hipSuccess) st = HLB_EDEVICE;
    if (st == HLB_OK) *out = h > (unsigned long long)INT64_MAX ? INT64_MAX : (int64_t)h;
    return st;
}

// Shared argument checks and plaintext bound of the CP-MM entry points.
static hlb_status cp_mm_prepare(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P, int64_t ldp,
                                int64_t *p_absmax, const uint64_t *A, const uint64_t *B, const uint64_t *primes,
                                int L, uint64_t *PA, uint64_t *PB, hipStream_t s, uint64_t *qmin, uint64_t *qmax,
                                int *n_xcd, bool *nothing) {
    *nothing = false;
    if (m < 0 || k < 0 || nA < 0 || nB < 0 || L < 0 || L > 1024 || *p_absmax < 0 ||
        (uint64_t)*p_absmax >= kMaxModulus)
        return HLB_EINVAL;
    if (L == 0 || m == 0 || (nA == 0 && nB == 0)) {
        *nothing = true;
        return HLB_OK;
    }
    if (!primes) return HLB_EINVAL;
    *qmin = UINT64_MAX;
    *qmax = 0;
    for (int l = 0; l < L; ++l) {
        if (check_modulus(primes[l]) != HLB_OK) return HLB_EINVAL;
        *qmax = std::max(*qmax, primes[l]);
        *qmin = std::min(*qmin, primes[l]);
    }
    if ((nA > 0 && !PA) || (nB > 0 && !PB)) return HLB_EINVAL;
    if (k > 0 && (!P || ldp < k || (nA > 0 && !A) || (nB > 0 && !B))) return HLB_EINVAL;
    hlb_status st = device_ready(n_xcd);
    if (st != HLB_OK) return st;
    if (*p_absmax == 0 && k > 0) {
        if ((st = measure_absmax(P, m, k, ldp, p_absmax, s)) != HLB_OK) return st;
        if ((uint64_t)*p_absmax >= kMaxModulus) return HLB_ERANGE;
    }
    return HLB_OK;
}

hlb_status cp_mm_entry(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P, int64_t ldp, int64_t p_absmax,
                       const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L, uint64_t *PA, uint64_t *PB,
                       int form, hipStream_t s) {
    uint64_t qmin = 0, qmax = 0;
    int n_xcd = 8;
    bool nothing = false;
    hlb_status st = cp_mm_prepare(m, k, nA, nB, P, ldp, &p_absmax, A, B, primes, L, PA, PB, s, &qmin, &qmax,
                                  &n_xcd, &nothing);
    if (st != HLB_OK || nothing) return st;
    form = resolve_form(form);
    Plan pl;
    if ((st = plan(1, k, qmax, std::max<int64_t>(p_absmax, 1), form, &pl)) != HLB_OK) return st;
    auto_for_shape(&pl, form, m, std::max(nA, nB), k, qmax, std::max<int64_t>(p_absmax, 1));
    choose_class(&pl, m, std::max(nA, nB), k);
    std::vector<RightSpec> rights;
    LeftSpec left{P, ldp, m, {}, {}};
    for (int l = 0; l < L; ++l) {
        if (nA > 0) {
            rights.push_back({A + (int64_t)l * k * nA, nA, nA, primes[l]});
            left.C.push_back(PA + (int64_t)l * m * nA);
            left.ldc.push_back(nA);
        }
        if (nB > 0) {
            rights.push_back({B + (int64_t)l * k * nB, nB, nB, primes[l]});
            left.C.push_back(PB + (int64_t)l * m * nB);
            left.ldc.push_back(nB);
        }
    }
    return run_products(pl, {left}, rights, k, n_xcd, s);
}

// The input checks of HLB_OPT_VALIDATE for one CP-MM (synchronous; HLB_EINVAL on a capturing
// stream): every residue of A and B below its prime, every |P| within p_absmax (when one is
// given).  HLB_ERANGE on the first violation; arguments the call itself refuses pass here.
hlb_status validate_cp_mm(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P, int64_t ldp,
                          int64_t p_absmax, const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L,
                          void *stream) {
    if (m <= 0 || k <= 0 || L <= 0 || L > 1024 || !primes || (nA <= 0 && nB <= 0) || !P || ldp < k) return HLB_OK;
    if ((nA > 0 && !A) || (nB > 0 && !B)) return HLB_OK;
    int64_t bad = -1;
    for (int l = 0; l < L; ++l) {
        if (check_modulus(primes[l]) != HLB_OK) return HLB_OK;
        hlb_status v = HLB_OK;
        if (nA > 0) v = hlb_validate_residues(A + (int64_t)l * k * nA, k, nA, nA, primes[l], &bad, stream);
        if (v == HLB_OK && nB > 0) v = hlb_validate_residues(B + (int64_t)l * k * nB, k, nB, nB, primes[l], &bad, stream);
        if (v != HLB_OK) return v;
    }
    if (p_absmax > 0) {
        int64_t mx = 0;
        const hlb_status v = hlb_plaintext_absmax(P, m, k, ldp, &mx, stream);
        if (v != HLB_OK) return v;
        if (mx > p_absmax) return HLB_ERANGE;
    }
    return HLB_OK;
}

}  // namespace hlb

using namespace hlb;

// ===========================================================================================
// extern "C" entry points
// ===========================================================================================
extern "C" {

const char *hlb_status_str(int s) {
    switch (s) {
        case HLB_OK: return "ok";
        case HLB_EINVAL: return "invalid argument";
        case HLB_ERANGE: return "input entry out of range";
        case HLB_EBOUND: return "no exact limb plan for this form and shape";
        case HLB_ENOMEM: return "device workspace allocation failed";
        case HLB_EDEVICE: return "HIP runtime or kernel launch failure";
        case HLB_EUNSUP: return "unsupported device or option";
        case HLB_ESCRATCH: return "workspace exceeds the no-allocation scratch buffer";
        default: return "unknown status";
    }
}

hlb_status hlb_plan(int kind, int64_t k, uint64_t q_max, int64_t p_absmax, int form, hlb_plan_desc *out) {
    if (!out || (kind != 0 && kind != 1) || k < 0 || check_modulus(q_max) != HLB_OK) return HLB_EINVAL;
    if (kind == 1 && (p_absmax < 1 || (uint64_t)p_absmax >= kMaxModulus)) return HLB_EINVAL;
    Plan pl;
    const hlb_status st = plan(kind, k, q_max, p_absmax, resolve_form(form), &pl);
    if (st != HLB_OK) return st;
    out->form = pl.form;
    out->p_limbs = pl.np;
    out->x_limbs = pl.nx;
    out->shifts = pl.np + pl.nx - 1;
    out->limb_bits = pl.limb_bits;
    out->max_pairs = pl.pairs;
    out->k_chunk = pl.kchunk;
    out->acc_bound_log2 = pl.acc_bound_log2;
    return HLB_OK;
}

hlb_status hlb_mod_pp_mm(uint64_t q, int64_t m, int64_t k, int64_t n, const uint64_t *P, int64_t ldp,
                         const uint64_t *X, int64_t ldx, uint64_t *C, int64_t ldc, int form, void *stream) {
    if (check_modulus(q) != HLB_OK || m < 0 || k < 0 || n < 0) return HLB_EINVAL;
    if (m == 0 || n == 0) return HLB_OK;
    if (!C || ldc < n || (k > 0 && (!P || !X || ldp < k || ldx < n))) return HLB_EINVAL;
    form = resolve_form(form);
    if (opt_validate() && k > 0) {
        int64_t bad = -1;
        hlb_status v = hlb_validate_residues(P, m, k, ldp, q, &bad, stream);
        if (v == HLB_OK) v = hlb_validate_residues(X, k, n, ldx, q, &bad, stream);
        if (v != HLB_OK) return v;
    }
    Plan pl;
    hlb_status st = plan(0, k, q, 0, form, &pl);
    if (st != HLB_OK) return st;
    auto_for_shape(&pl, form, m, n, k, q, 0);
    choose_class(&pl, m, n, k);
    int n_xcd = 8;
    if ((st = device_ready(&n_xcd)) != HLB_OK) return st;
    std::vector<RightSpec> rights{{X, ldx, n, q}};
    std::vector<LeftSpec> lefts{{(const int64_t *)P, ldp, m, {C}, {ldc}}};
    return run_products(pl, lefts, rights, k, n_xcd, (hipStream_t)stream);
}

hlb_status hlb_cp_mm(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P, int64_t ldp,
                     int64_t p_absmax, const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L,
                     uint64_t *PA, uint64_t *PB, int form, void *stream) {
    if (opt_validate()) {
        const hlb_status v = validate_cp_mm(m, k, nA, nB, P, ldp, p_absmax, A, B, primes, L, stream);
        if (v != HLB_OK) return v;
    }
    return cp_mm_entry(m, k, nA, nB, P, ldp, p_absmax, A, B, primes, L, PA, PB, form, (hipStream_t)stream);
}

hlb_status hlb_plan_trunc_b(int64_t k, uint64_t q_min, uint64_t q_max, int64_t p_absmax, double b_err_log2,
                            int form, hlb_trunc_desc *out) {
    if (!out || k < 0 || check_modulus(q_min) != HLB_OK || check_modulus(q_max) != HLB_OK || q_min > q_max ||
        p_absmax < 1 || (uint64_t)p_absmax >= kMaxModulus)
        return HLB_EINVAL;
    Plan pl;
    const hlb_status st = plan_trunc_b(k, q_min, q_max, p_absmax, b_err_log2, form, &pl);
    if (st != HLB_OK) return st;
    out->form = pl.form;
    out->truncated = pl.drop > 0 || pl.trunc;
    out->dropped_shifts = pl.drop;
    int products = pl.np * pl.nx;
    for (int i = 0; i < pl.np; ++i)
        for (int j = 0; j < pl.nx; ++j)
            if (i + j < pl.drop) --products;
    out->products = products;
    out->err_bound_log2 = pl.err_bound_log2;
    return HLB_OK;
}

hlb_status hlb_cp_mm_trunc_b(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P, int64_t ldp,
                             int64_t p_absmax, const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L,
                             uint64_t *PA, uint64_t *PB, double b_err_log2, int form, void *stream) {
    const hipStream_t s = (hipStream_t)stream;
    uint64_t qmin = 0, qmax = 0;
    int n_xcd = 8;
    bool nothing = false;
    // one modulus only: over an RNS basis every prime's product would carry its own error,
    // and the CRT lift of such residues is not close to the exact product
    if (L > 1) return HLB_EINVAL;
    hlb_status st = cp_mm_prepare(m, k, nA, nB, P, ldp, &p_absmax, A, B, primes, L, PA, PB, s, &qmin, &qmax,
                                  &n_xcd, &nothing);
    if (st != HLB_OK || nothing) return st;
    const int64_t pmax = std::max<int64_t>(p_absmax, 1);
    Plan pa, pb;
    if ((st = plan(1, k, qmax, pmax, form, &pa)) != HLB_OK) return st;
    if ((st = plan_trunc_b(k, qmin, qmax, pmax, b_err_log2, form, &pb)) != HLB_OK) return st;
    auto_for_shape(&pa, form, m, std::max(nA, nB), k, qmax, pmax);
    if (!pb.trunc && pb.drop == 0) auto_for_shape(&pb, form, m, std::max(nA, nB), k, qmax, pmax);
    choose_class(&pa, m, std::max(nA, nB), k);
    choose_class(&pb, m, std::max(nA, nB), k);
    LeftSpec la{P, ldp, m, {}, {}}, lb{P, ldp, m, {}, {}};
    std::vector<RightSpec> ra, rb;
    for (int l = 0; l < L; ++l) {
        if (nA > 0) {
            ra.push_back({A + (int64_t)l * k * nA, nA, nA, primes[l]});
            la.C.push_back(PA + (int64_t)l * m * nA);
            la.ldc.push_back(nA);
        }
        if (nB > 0) {
            rb.push_back({B + (int64_t)l * k * nB, nB, nB, primes[l]});
            lb.C.push_back(PB + (int64_t)l * m * nB);
            lb.ldc.push_back(nB);
        }
    }
    if (!pb.trunc && pb.drop == 0) {
        // nothing truncated: the exact CP-MM in one launch
        for (size_t i = 0; i < rb.size(); ++i) {
            ra.push_back(rb[i]);
            la.C.push_back(lb.C[i]);
            la.ldc.push_back(lb.ldc[i]);
        }
        return run_products(pa, {la}, ra, k, n_xcd, s);
    }
    if ((st = run_products(pa, {la}, ra, k, n_xcd, s)) != HLB_OK) return st;
    return run_products(pb, {lb}, rb, k, n_xcd, s);
}

hlb_status hlb_ccmm_pp_core(int64_t m, int64_t k, int64_t n, const uint64_t *A, const uint64_t *B,
                            const uint64_t *At, const uint64_t *Bt, const uint64_t *primes, int L,
                            uint64_t *C00, uint64_t *C01, uint64_t *C10, uint64_t *C11, int form, void *stream) {
    if (m < 0 || k < 0 || n < 0 || L < 0 || L > 1024) return HLB_EINVAL;
    if (L == 0 || m == 0 || n == 0) return HLB_OK;
    if (!primes || !C00 || !C01 || !C10 || !C11) return HLB_EINVAL;
    if (k > 0 && (!A || !B || !At || !Bt)) return HLB_EINVAL;
    uint64_t qmax = 0;
    for (int l = 0; l < L; ++l) {
        if (check_modulus(primes[l]) != HLB_OK) return HLB_EINVAL;
        qmax = std::max(qmax, primes[l]);
    }
    form = resolve_form(form);
    Plan pl;
    hlb_status st = plan(0, k, qmax, 0, form, &pl);
    if (st != HLB_OK) return st;
    auto_for_shape(&pl, form, m, n, k, qmax, 0);
    choose_class(&pl, m, n, k);
    int n_xcd = 8;
    if ((st = device_ready(&n_xcd)) != HLB_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    for (int l = 0; l < L; ++l) {
        const int64_t om = (int64_t)l * m * n, ia = (int64_t)l * m * k, ix = (int64_t)l * k * n;
        // both right operands split once, each left operand split once (run_products)
        std::vector<RightSpec> rights{{At + ix, n, n, primes[l]}, {Bt + ix, n, n, primes[l]}};
        std::vector<LeftSpec> lefts{{(const int64_t *)(A + ia), k, m, {C00 + om, C01 + om}, {n, n}},
                                    {(const int64_t *)(B + ia), k, m, {C10 + om, C11 + om}, {n, n}}};
        if ((st = run_products(pl, lefts, rights, k, n_xcd, s)) != HLB_OK) return st;
    }
    return HLB_OK;
}

hlb_status hlb_rescale(int64_t count, const uint64_t *X, const uint64_t *primes, int L, uint64_t *Y, void *stream) {
    if (count < 0 || L < 2 || L > kMaxRescalePrimes || !primes) return HLB_EINVAL;
    RescaleConsts rc;
    std::memset(&rc, 0, sizeof(rc));
    rc.L = L;
    const uint64_t q = primes[L - 1];
    for (int l = 0; l < L; ++l) {
        if (check_modulus(primes[l]) != HLB_OK) return HLB_EINVAL;
        rc.q[l] = primes[l];
    }
    for (int l = 0; l < L - 1; ++l) {
        const uint64_t ql = primes[l];
        rc.q_mod[l] = q % ql;
        // q^{-1} mod ql by the extended Euclidean algorithm (signed 128-bit)
        __int128 r0 = (__int128)ql, r1 = (__int128)(q % ql), t0 = 0, t1 = 1;
        while (r1 != 0) {
            const __int128 qt = r0 / r1, r2 = r0 - qt * r1, t2 = t0 - qt * t1;
            r0 = r1;
            r1 = r2;
            t0 = t1;
            t1 = t2;
        }
        if (r0 != 1) return HLB_EINVAL;  // not invertible
        if (t0 < 0) t0 += ql;
        rc.qinv[l] = (uint64_t)t0;
        rc.qinv_shoup[l] = (uint64_t)(((unsigned __int128)rc.qinv[l] << 64) / ql);
    }
    if (count == 0) return HLB_OK;
    if (!X || !Y) return HLB_EINVAL;
    hlb_status st = device_ready(nullptr);
    if (st != HLB_OK) return st;
    return launch_rescale(X, count, rc, Y, (hipStream_t)stream) == hipSuccess ? HLB_OK : HLB_EDEVICE;
}

hlb_status hlb_validate_residues(const uint64_t *X, int64_t rows, int64_t cols, int64_t ld, uint64_t q,
                                 int64_t *first_bad, void *stream) {
    if (!first_bad || rows < 0 || cols < 0 || q < 1) return HLB_EINVAL;
    *first_bad = -1;
    if (rows == 0 || cols == 0) return HLB_OK;
    if (!X || ld < cols) return HLB_EINVAL;
    hlb_status st = device_ready(nullptr);
    if (st != HLB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (stream_capturing(s)) return HLB_EINVAL;  // synchronous: not capturable
    unsigned long long *d = nullptr;
    if (hipMallocAsync((void **)&d, sizeof(*d), s) != hipSuccess) {
        (void)hipGetLastError();
        return HLB_ENOMEM;
    }
    unsigned long long h = ~0ull;
    if (launch_fill((uint64_t *)d, 1, 1, 1, ~(uint64_t)0, s) != hipSuccess) st = HLB_EDEVICE;
    if (st == HLB_OK && launch_validate(X, rows, cols, ld, q, d, s) != hipSuccess) st = HLB_EDEVICE;
    if (st == HLB_OK && hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) st = HLB_EDEVICE;
    (void)hipFreeAsync(d, s);
    if (hipStreamSynchronize(s) != hipSuccess) st = HLB_EDEVICE;
    if (st != HLB_OK) return st;
    if (h != ~0ull) {
        *first_bad = (int64_t)h;
        return HLB_ERANGE;
    }
    return HLB_OK;
}

hlb_status hlb_plaintext_absmax(const int64_t *P, int64_t m, int64_t k, int64_t ld, int64_t *absmax,
                                void *stream) {
    if (!absmax || m < 0 || k < 0) return HLB_EINVAL;
    *absmax = 0;
    if (m == 0 || k == 0) return HLB_OK;
    if (!P || ld < k) return HLB_EINVAL;
    hlb_status st = device_ready(nullptr);
    if (st != HLB_OK) return st;
    return measure_absmax(P, m, k, ld, absmax, (hipStream_t)stream);
}

hlb_status hlb_set_option(int option, int64_t value) {
    switch (option) {
        case HLB_OPT_FORCE_KCHUNK:
            if (value < 0) return HLB_EINVAL;
            g_force_kchunk.store(value);
            return HLB_OK;
        case HLB_OPT_PROFILE:
            g_profile.store(value ? 1 : 0);
            return HLB_OK;
        case HLB_OPT_BATCH_GRAPH:
            g_batch_graph.store(value ? 1 : 0);
            return HLB_OK;
        case HLB_OPT_FORCE_CLASS:
            if (value < -1 || value > 1) return HLB_EINVAL;
            g_force_class.store((int)value);
            return HLB_OK;
        case HLB_OPT_F64_PLANES:
            g_f64_planes.store(value ? 1 : 0);
            return HLB_OK;
        case HLB_OPT_CRT_WIDE:
            if (value < -1 || value > 2) return HLB_EINVAL;
            g_crt_wide.store((int)value);
            return HLB_OK;
        case HLB_OPT_WS_CAP:
            if (value < 0) return HLB_EINVAL;
            read_env();  // the option set here outlasts the environment's value
            g_ws_cap.store(value);
            return HLB_OK;
        case HLB_OPT_VALIDATE:
            read_env();  // the option set here outlasts the environment's value
            g_validate.store(value ? 1 : 0);
            return HLB_OK;
        default: return HLB_EUNSUP;
    }
}

hlb_status hlb_profile_read(const char *name, int64_t *launches, double *total_ms) {
    if (!name || !launches || !total_ms) return HLB_EINVAL;
    *launches = 0;
    *total_ms = 0.0;
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (ProfRec &r : g_prof) {
        if (r.name != name) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return HLB_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return HLB_EDEVICE;
        *launches += 1;
        *total_ms += ms;
    }
    return HLB_OK;
}

hlb_status hlb_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (ProfRec &r : g_prof) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    return HLB_OK;
}

hlb_status hlb_tune_set(int x_digits, int log2m, int log2n, int log2k, int cls) {
    if (x_digits < 1 || x_digits > 8 || log2m < 0 || log2m > 63 || log2n < 0 || log2n > 63 || log2k < 0 ||
        log2k > 63 || cls < -1 || cls > 1)
        return HLB_EINVAL;
    std::lock_guard<std::mutex> g(g_tune_mu);
    const uint32_t key = tune_key(x_digits, log2m, log2n, log2k);
    if (cls < 0) g_tune.erase(key);
    else g_tune[key] = cls;
    return HLB_OK;
}

hlb_status hlb_tune_set_crt(int moduli, int log2m, int log2n, int log2k, int cls) {
    if (moduli < 1 || moduli > kCrtMaxModuli || !tune_fields_ok(log2m, log2n, log2k) || cls < -1 || cls > 2)
        return HLB_EINVAL;
    std::lock_guard<std::mutex> g(g_tune_mu);
    const uint32_t key = tune_key_crt(moduli, log2m, log2n, log2k);
    if (cls < 0) g_tune.erase(key);
    else g_tune[key] = cls;
    return HLB_OK;
}

int hlb_tune_class_crt(int moduli, int64_t m, int64_t n, int64_t k) {
    if (moduli < 1 || moduli > kCrtMaxModuli || m < 1 || n < 1 || k < 1) return -1;
    return crt_tile_class(moduli, m, n, k);
}

hlb_status hlb_tune_load(const char *path) {
    if (!path) return HLB_EINVAL;
    std::lock_guard<std::mutex> g(g_tune_mu);
    return tune_load_locked(path);
}

int hlb_tune_class(int x_digits, int64_t m, int64_t n, int64_t k) {
    if (m < 1 || n < 1 || k < 1) return -1;
    Plan pl;
    pl.form = HLB_FORM_INT8;
    pl.np = 3;
    pl.nx = x_digits;
    const I8Shape sh = i8_shape(3, x_digits, 0);
    if (!sh.dp) return -1;
    choose_class(&pl, m, n, k);
    return pl.cls;
}

hlb_status hlb_release(void) {
    if (hipDeviceSynchronize() != hipSuccess) return HLB_EDEVICE;
    batch_release();
    ws_release_all();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HLB_EDEVICE;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    return HLB_OK;
}

// ------------------------------- test-only helpers --------------------------------------

hlb_status hlb_test_encode(const double *M, int64_t count, double delta, int64_t *out, void *stream) {
    if (count < 0 || (count > 0 && (!M || !out))) return HLB_EINVAL;
    if (count == 0) return HLB_OK;
    hlb_status st = device_ready(nullptr);
    if (st != HLB_OK) return st;
    return launch_encode(M, count, delta, out, (hipStream_t)stream) == hipSuccess ? HLB_OK : HLB_EDEVICE;
}

// B[l] = -(A[l] S) + Menc mod q_l, or D[l] = A[l] S + B[l]: one Mod-PP-MM with the residue
// matrix A on the left and the small signed S (mapped to residues) on the right.
static hlb_status test_linear(int64_t rows, int64_t n, const uint64_t *A, const int64_t *S, const int64_t *Es,
                              const uint64_t *Eu, int sign, const uint64_t *primes, int L, uint64_t *out,
                              hipStream_t s) {
    if (rows < 0 || n < 0 || L < 0 || (L > 0 && !primes)) return HLB_EINVAL;
    if (rows == 0 || n == 0 || L == 0) return HLB_OK;
    if (!A || !S || !out || (!Es && !Eu)) return HLB_EINVAL;
    for (int l = 0; l < L; ++l)
        if (check_modulus(primes[l]) != HLB_OK) return HLB_EINVAL;
    hlb_status st = device_ready(nullptr);
    if (st != HLB_OK) return st;
    void *Sres = nullptr, *AS = nullptr;
    if ((st = ws_alloc(&Sres, (size_t)(n * n * 8), s)) != HLB_OK) return st;
    if ((st = ws_alloc(&AS, (size_t)(rows * n * 8), s)) != HLB_OK) {
        ws_free(Sres, s);
        return st;
    }
    for (int l = 0; l < L && st == HLB_OK; ++l) {
        const uint64_t q = primes[l];
        if (launch_residues_of_signed(S, n * n, q, (uint64_t *)Sres, s) != hipSuccess) {
            st = HLB_EDEVICE;
            break;
        }
        st = hlb_mod_pp_mm(q, rows, n, n, A + (int64_t)l * rows * n, n, (const uint64_t *)Sres, n,
                           (uint64_t *)AS, n, HLB_FORM_AUTO, s);
        if (st != HLB_OK) break;
        if (launch_combine((const uint64_t *)AS, Es, Eu ? Eu + (int64_t)l * rows * n : nullptr, sign, rows * n, q,
                           out + (int64_t)l * rows * n, s) != hipSuccess)
            st = HLB_EDEVICE;
    }
    ws_free(Sres, s);
    ws_free(AS, s);
    return st;
}

hlb_status hlb_test_encrypt(int64_t k, int64_t n, const uint64_t *A, const int64_t *S, const int64_t *Menc,
                            const uint64_t *primes, int L, uint64_t *B, void *stream) {
    return test_linear(k, n, A, S, Menc, nullptr, -1, primes, L, B, (hipStream_t)stream);
}

hlb_status hlb_test_decrypt(int64_t rows, int64_t n, const uint64_t *A, const uint64_t *B, const int64_t *S,
                            const uint64_t *primes, int L, uint64_t *D, void *stream) {
    return test_linear(rows, n, A, S, nullptr, B, +1, primes, L, D, (hipStream_t)stream);
}

}  // extern "C"
