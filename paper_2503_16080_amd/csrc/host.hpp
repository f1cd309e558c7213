// host.hpp -- internal host-side interfaces of libhlb (planner, dispatch, profiling).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hlb.h"
#include "common.hpp"

namespace hlb {

// An exact limb plan: limb counts, bits per limb and the K chunk that keeps every
// accumulator inside the exact range of its type (Lemma le:strategy1).
struct Plan {
    int form = 0;
    int kind = 1;           // 0: both operands residues (Mod-PP-MM); 1: signed plaintext on the left
    int np = 0, nx = 0;     // limbs of the left / right operand (instantiated counts); CRT: moduli
    int limb_bits = 0;
    int pairs = 0;          // most limb products sharing one accumulator
    int64_t kchunk = 0;     // K elements accumulated before a fold
    int bm = 0, bn = 0, bk = 0;
    int cls = 0;            // INT8 tile class (0: 128 x 64, 1: 64 x 128)
    double acc_bound_log2 = 0.0;
    // Truncated plans (Strategy 2 of Section 6.1), only for the b-part of a CP-MM:
    int drop = 0;           // INT8: digit products of shifts < drop are skipped
    bool trunc = false;     // FP64: one product of the rounded operands
    double err_bound_log2 = -__builtin_inf();  // worst-case |result - exact| (centred), log2
};

// Cheapest b-part plan in `form` whose worst-case error is at most 2^err_log2 (and below
// q_min / 2); the exact plan always qualifies.
hlb_status plan_trunc_b(int64_t k, uint64_t qmin, uint64_t qmax, int64_t pmax, double err_log2, int form, Plan *pl);

hlb_status plan(int kind, int64_t k, uint64_t qmax, int64_t pmax, int form, Plan *pl);

// Operands of run_products: left operands (plaintexts or residue matrices, m x k) and right
// operands (residue matrices, k x n, each with its modulus); C[r] / ldc[r] of a left operand
// receive its product with right operand r.
struct LeftSpec {
    const int64_t *P;
    int64_t ldp, m;
    std::vector<uint64_t *> C;
    std::vector<int64_t> ldc;
};
struct RightSpec {
    const uint64_t *X;
    int64_t ldx, n;
    uint64_t q;
};
hlb_status run_products(const Plan &pl, const std::vector<LeftSpec> &lefts, const std::vector<RightSpec> &rights,
                        int64_t k, int n_xcd, hipStream_t s);
// Picks the INT8 tile class of a problem (m rows, n columns per output matrix, depth k) and
// updates pl->cls / bm / bn accordingly; no-op for plans with a single class.
void choose_class(Plan *pl, int64_t m, int64_t n, int64_t k);
// The multimodular GEMM's tile class (0: 256 x 128, 1: 256 x 256, 2: 256 x 384 outputs) for D
// moduli, m rows, n columns per output matrix and depth k: forced by HLB_OPT_CRT_WIDE, else
// from the tuning table, else 2.
int crt_tile_class(int D, int64_t m, int64_t n, int64_t k);
int i8_digits_for(uint64_t vmax);
hlb_status check_modulus(uint64_t q);
hlb_status device_ready(int *n_xcd, int *cus = nullptr);
void fill_seg(Seg &s, uint64_t q, int limb_bits);
hlb_status ws_alloc(void **p, size_t bytes, hipStream_t s);
void ws_free(void *p, hipStream_t s);
void ws_release_all();

// The workspace of one call: n buffers carved, 256-byte aligned, from one block kept with the
// call's stream (device, stream) and reused by the next call on it.  Calls on one stream run in
// stream order, so the block is free again once a call is enqueued; the lease also holds the
// stream's block against concurrent calls from other host threads until it is destroyed.  The
// block grows to the largest workspace a call on the stream has needed (ws_release_all returns
// it).  Under graph capture the buffers come from the pool instead, owned by the graph.
struct WsSlot;
class WsLease {
  public:
    WsLease() = default;
    WsLease(const WsLease &) = delete;
    WsLease &operator=(const WsLease &) = delete;
    ~WsLease();
    // HLB_ENOMEM when a buffer is above the workspace cap or the block cannot grow.
    hlb_status take(hipStream_t s, const size_t *bytes, void **ptrs, int n);

  private:
    WsSlot *slot_ = nullptr;
    void *own_ = nullptr;
    hipStream_t s_ = nullptr;
};
// While alive, WsLease::take on this thread carves every workspace from [base, base + bytes)
// instead of allocating, and returns HLB_ESCRATCH when a call needs more.
class ScratchScope {
  public:
    ScratchScope(void *base, size_t bytes);
    ~ScratchScope();
    ScratchScope(const ScratchScope &) = delete;
    ScratchScope &operator=(const ScratchScope &) = delete;
    void *base() const { return base_; }
    size_t bytes() const { return bytes_; }

  private:
    void *base_;
    size_t bytes_;
    const ScratchScope *prev_;
};

// hlb_cp_mm's work (argument checks, plan, products) on stream s.
hlb_status cp_mm_entry(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P, int64_t ldp, int64_t p_absmax,
                       const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L, uint64_t *PA, uint64_t *PB,
                       int form, hipStream_t s);
// HLB_OPT_VALIDATE's checks of one CP-MM's inputs (synchronous; HLB_ERANGE on a violation).
hlb_status validate_cp_mm(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P, int64_t ldp,
                          int64_t p_absmax, const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L,
                          void *stream);
// The form a call runs: `form`, or the HLB_FORM environment's form where `form` is
// HLB_FORM_AUTO.
int resolve_form(int form);
bool opt_validate();
int64_t opt_force_kchunk();
bool opt_batch_graph();
void batch_release();

// Brackets a kernel launch with HIP events on its stream while profiling is enabled.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();

  private:
    std::string name_;
    hipStream_t stream_;
    hipEvent_t a_{}, b_{};
    bool active_ = false;
};

}  // namespace hlb
