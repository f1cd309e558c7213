/*
 * hlb.h -- C ABI of libhlb: bit-exact ciphertext-plaintext matrix products (CP-MM) for CKKS
 * on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the reduction of CP-MM to modular plaintext matrix products
 * (Mod-PP-MM) over each RNS prime (Algorithm alg:pcmm step 1; Theorems th:pcmm and
 * th:pcmm-shs), and evaluates every Mod-PP-MM exactly, in one of three forms (Section 6.1):
 *   HLB_FORM_INT8_CRT  Strategy 3 (FLINT variant): the centred integer product modulo small
 *                      coprime moduli <= 256, one INT8->INT32 matrix product each, then the CRT;
 *   HLB_FORM_INT8      Strategy 1 with balanced signed 8-bit digits on the INT8 matrix cores;
 *   HLB_FORM_FP64      Strategy 1 with 17..26-bit limbs on the FP64 matrix cores (the
 *                      paper's form).
 * All produce the unique canonical result in [0, q) -- bit-identical to each other.
 * hlb_cp_mm_trunc_b adds Strategy 2 (an approximate b-part) over one modulus.
 *
 * Orientation.  The paper multiplies an encrypted matrix on the right, M * U.  This ABI takes
 * the plaintext on the LEFT, C = P * X, which is the same computation on transposed
 * matrices; a ciphertext (A, B) satisfying the row identity A * S + B = Delta * M (mod q)
 * (Eq mat_row_format) is mapped by left multiplication to (P A, P B), an encryption of P M.
 *
 * Conventions for every entry point:
 *  - Matrices are row-major.  "ld" arguments are row strides in ELEMENTS (>= row length).
 *  - Matrix pointers are DEVICE pointers owned by the caller; the library never frees them.
 *    Prime lists, problem tables and result scalars are HOST pointers.
 *  - Residues are uint64 values in [0, q).  Plaintext matrices are signed int64.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Product calls only
 *    enqueue work on it and return; results are ready when the stream is synchronised.
 *    Argument and planning errors are reported synchronously, before anything is enqueued.
 *    Entry points documented as "synchronous" synchronise `stream` before returning.
 *  - Moduli: 2 <= q < 2^52.
 *  - Workspace (digit or residue planes, the multimodular bytes, FP64 double planes) comes
 *    from one device block the library keeps per (device, stream): each call carves its
 *    buffers from its stream's block, which grows to the largest workspace a call on that
 *    stream has needed and is reused by the next call in stream order.  Concurrent calls on
 *    one stream from several host threads take turns on the block.  Under graph capture the
 *    workspace is a stream-ordered pool allocation owned by the graph.  hlb_release()
 *    returns every block; a destroyed stream's block is kept until then, so a stream must
 *    have finished its library work before it is destroyed.
 *  - Calls on different streams may run concurrently.
 *  - The functions are not re-entrant during hlb_release().
 */
#ifndef HLB_H
#define HLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HLB_OK = 0,
    HLB_EINVAL = 1,  /* bad shape, null pointer, leading dimension, count or modulus */
    HLB_ERANGE = 2,  /* an input entry lies outside its stated range (checked entry points) */
    HLB_EBOUND = 3,  /* no exact limb plan exists for this form, shape and input bound */
    HLB_ENOMEM = 4,  /* device workspace allocation failed */
    HLB_EDEVICE = 5, /* a HIP runtime call or kernel launch failed */
    HLB_EUNSUP = 6,  /* device is not gfx950, or the requested option is unknown */
    HLB_ESCRATCH = 7 /* hlb_cp_mm_noalloc: the call needs more workspace than its static
                        scratch buffer holds (HLB_NOALLOC_SCRATCH_BYTES) */
} hlb_status;

typedef enum {
    HLB_FORM_AUTO = 0,     /* multimodular where it needs under 3/4 of the digit products
                              (and m, n >= 256), else INT8 digits, else FP64 */
    HLB_FORM_FP64 = 1,     /* FP64 limbs on v_mfma_f64_16x16x4_f64 */
    HLB_FORM_INT8 = 2,     /* balanced int8 digits on v_mfma_i32_32x32x32_i8 (Strategy 1);
                              every k up to 4.79 million runs; deeper K may be refused with
                              HLB_EINVAL (the tiles address their digit panels with 32-bit
                              offsets: K blocks x panel bytes per block must stay below 2^32) */
    HLB_FORM_INT8_CRT = 3  /* multimodular: the centred integer product modulo D coprime
                              moduli <= 256, one int8 GEMM each, recombined by the CRT
                              (Strategy 3, FLINT variant); needs k <= 131071 */
} hlb_form;

/* Human-readable name of a status code (static string, never NULL). */
const char *hlb_status_str(int status);

/*
 * Mod-PP-MM_{q; m,k,n} (Section 5 notation): C = P * X mod q.
 *   P: m x k residues in [0, q) (row stride ldp >= k), X: k x n residues (ldx >= n),
 *   C: m x n output, written with canonical residues in [0, q) (ldc >= n).
 * m == 0 or n == 0 is a no-op; k == 0 writes zeros.  Inputs >= q violate the precondition
 * (the result is then unspecified but the call stays memory-safe); check them with
 * hlb_validate_residues.  C must not alias P or X.
 */
hlb_status hlb_mod_pp_mm(uint64_t q, int64_t m, int64_t k, int64_t n,
                         const uint64_t *P, int64_t ldp, const uint64_t *X, int64_t ldx,
                         uint64_t *C, int64_t ldc, int form, void *stream);

/*
 * CP-MM over L RNS primes (Algorithm alg:pcmm step 1 without the Rescale; Theorem
 * th:pcmm-shs: two Mod-PP-MMs per modulus):
 *     PA[l] = P * A[l] mod primes[l],   PB[l] = P * B[l] mod primes[l],   l < L.
 *   P:  m x k signed plaintext (ldp >= k) with every |P[i][j]| <= p_absmax.
 *       The same P serves all primes and both parts: it is split into digits once.
 *   p_absmax: a bound on |P| (1 <= p_absmax < 2^52).  Pass 0 to have the library measure
 *       it on the device (that makes the call synchronous, and on a stream under graph
 *       capture it is refused with HLB_EINVAL before anything is enqueued).
 *   A:  [L][k][nA] residues, dense (prime l's matrix at A + l*k*nA); B: [L][k][nB].
 *   PA: [L][m][nA] output, dense; PB: [L][m][nB] output, dense.
 *   primes: host array of L moduli, each 2 <= q < 2^52.
 * L == 0, m == 0 or nA == nB == 0 are no-ops.  |P| > p_absmax violates the precondition.
 */
hlb_status hlb_cp_mm(int64_t m, int64_t k, int64_t nA, int64_t nB,
                     const int64_t *P, int64_t ldp, int64_t p_absmax,
                     const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L,
                     uint64_t *PA, uint64_t *PB, int form, void *stream);

/*
 * hlb_cp_mm for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Same arguments, results and forms
 * as hlb_cp_mm, bit-identical to it, with two differences:
 *   - Every workspace buffer (operand planes, multimodular product bytes, FP64 planes) is
 *     carved from one static device array of HLB_NOALLOC_SCRATCH_BYTES, which each device the
 *     library runs on holds from the library's first use there until the process ends.  The
 *     call allocates and frees nothing.  A call whose workspace exceeds the array returns
 *     HLB_ESCRATCH before anything is enqueued (about d = 1024 over 3 primes fits in every
 *     form; hlb_cp_mm has no such limit).
 *   - p_absmax must be given (>= 1): measuring it would allocate (HLB_EINVAL for 0).
 * The array is shared by every hlb_cp_mm_noalloc call on a device and keeps the last call's
 * contents (nothing in it needs clearing: every call writes all the bytes it reads).  Calls
 * on one stream run in stream order; calls that overlap on one device (different streams,
 * concurrent graph replays) race on the array and must be ordered by the caller.
 */
#define HLB_NOALLOC_SCRATCH_BYTES ((uint64_t)256 << 20)
hlb_status hlb_cp_mm_noalloc(int64_t m, int64_t k, int64_t nA, int64_t nB,
                             const int64_t *P, int64_t ldp, int64_t p_absmax,
                             const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L,
                             uint64_t *PA, uint64_t *PB, int form, void *stream);

/*
 * CP-MM with an approximate b-part (Strategy 2 of Section 6.1, "truncation") over ONE
 * modulus q = primes[0] (L must be 1): PA = P * A mod q exactly, as in hlb_cp_mm, and every
 * entry of PB equals the exact residue plus an integer e with |e| <= 2^b_err_log2
 * (PB = P * B + e mod q).  An error on the b-part reaches the decrypted message
 * unamplified (Section 6.1).  The method's error argument holds for a single modulus, the
 * paper's setting of one word-size q: over an RNS basis each prime's product would carry a
 * different error, and the CRT lift of such residues is not close to the exact product, so
 * L > 1 is rejected (HLB_EINVAL).  Other arguments as for hlb_cp_mm.
 *
 * The library takes the cheapest b-part plan of `form` whose worst-case error bound is at
 * most 2^b_err_log2 and below q / 2; the exact plan always qualifies:
 *   INT8: the digit products P_i B_j of the shifts i + j < drop (drop <= 3) are skipped:
 *         |e| <= k * 2^14 * sum_{s < drop} pairs(s) * 256^s, with pairs(s) the number of
 *         digit pairs of shift s.  Only when k needs no K fold (k <= 43690).
 *   FP64: one FP64 product of P and B rounded to doubles (B in its centred representative
 *         in (-q/2, q/2]), reduced mod q: |e| <= (k + 2) 2^-52 * k * p_absmax * (q/2)
 *         (zero when k * p_absmax * (q/2) < 2^53).  Needs k * p_absmax <= 2^51.
 * hlb_plan_trunc_b reports the choice.  The two parts are computed in separate launches.
 */
hlb_status hlb_cp_mm_trunc_b(int64_t m, int64_t k, int64_t nA, int64_t nB,
                             const int64_t *P, int64_t ldp, int64_t p_absmax,
                             const uint64_t *A, const uint64_t *B, const uint64_t *primes, int L,
                             uint64_t *PA, uint64_t *PB, double b_err_log2, int form, void *stream);

/* The b-part plan hlb_cp_mm_trunc_b takes for depth k, moduli in [q_min, q_max], |P| <=
 * p_absmax (>= 1) and budget b_err_log2. */
typedef struct {
    int form;             /* HLB_FORM_INT8 or HLB_FORM_FP64 */
    int truncated;        /* 0: the exact plan */
    int dropped_shifts;   /* INT8: shifts whose digit products are skipped */
    int products;         /* limb products per mod-q MAC of the b-part */
    double err_bound_log2;/* log2 of the worst-case |e|; -inf when exact */
} hlb_trunc_desc;
hlb_status hlb_plan_trunc_b(int64_t k, uint64_t q_min, uint64_t q_max, int64_t p_absmax,
                            double b_err_log2, int form, hlb_trunc_desc *out);

/*
 * The plaintext-product core of the ciphertext-ciphertext product (Algorithm alg:ccmm, step
 * 2): for every prime l < L, the four Mod-PP-MMs
 *     C00[l] = A[l] At[l],  C01[l] = A[l] Bt[l],  C10[l] = B[l] At[l],  C11[l] = B[l] Bt[l]
 * (mod primes[l]), i.e. [A; B] * [At Bt], with both operands full residues.  Each operand is
 * split into digits once and shared by the two products it enters.
 *   A, B:   [L][m][k] residues, dense;  At, Bt: [L][k][n] residues, dense;
 *   C00, C01, C10, C11: [L][m][n] outputs, dense.
 * The transposes, relinearisation and rescaling around this step are not part of the call.
 */
hlb_status hlb_ccmm_pp_core(int64_t m, int64_t k, int64_t n, const uint64_t *A, const uint64_t *B,
                            const uint64_t *At, const uint64_t *Bt, const uint64_t *primes, int L,
                            uint64_t *C00, uint64_t *C01, uint64_t *C10, uint64_t *C11, int form,
                            void *stream);

/*
 * Rescale by the last RNS prime (the Rescale step of Algorithm alg:pcmm, with the scaling
 * factor equal to the dropped prime, which then divides the modulus as Section 5 assumes):
 * for an integer x given by its residues X[l] = x mod primes[l], l < L, returns the residues
 * of floor(x / q + 1/2), q = primes[L-1], modulo each of the first L-1 primes:
 *     Y[l] = (x - c) * q^{-1} mod primes[l],   c = the representative of x mod q in
 *     (-q/2, q/2] (ties at q/2 taken upward),
 * which is exact and independent of the representative of x modulo the product of primes.
 *   X: [L][count] residues (count = rows * cols of each matrix, dense), Y: [L-1][count].
 * Requires L >= 2 and primes[L-1] invertible modulo every other prime (HLB_EINVAL if not).
 */
hlb_status hlb_rescale(int64_t count, const uint64_t *X, const uint64_t *primes, int L, uint64_t *Y,
                       void *stream);

/* One CP-MM of a batch: the fields mean what the hlb_cp_mm arguments of the same names
 * mean (dense layouts [L][k][nA], [L][k][nB], [L][m][nA], [L][m][nB]; P row stride ldp). */
typedef struct {
    int64_t m, k, nA, nB;
    const int64_t *P;
    int64_t ldp;
    int64_t p_absmax;
    const uint64_t *A, *B;
    uint64_t *PA, *PB;
} hlb_cpmm_problem;

/*
 * A batch of independent CP-MMs of uneven shapes that share the L primes (Theorem
 * th:pcmm-shs applied to each problem; the per-prime products are independent, as in
 * Section 6.1 Strategy 3).
 *   form HLB_FORM_INT8 or HLB_FORM_AUTO (plaintexts within 3 digits, primes within 7): all
 *     products run in ONE persistent kernel launch that pulls output tiles from a work list
 *     (largest first), preceded by one digit-split launch for all plaintexts and one for all
 *     ciphertext parts.
 *   form HLB_FORM_INT8_CRT: one residue-split launch for every operand, one GEMM launch over
 *     every (problem, modulus, tile) and one recombination launch, with the moduli count
 *     planned for the largest K and plaintext bound of the batch.
 *   other forms and plans run problem by problem through hlb_cp_mm.
 * The launch sequence is captured once per distinct batch signature (shapes, pointers,
 * primes, form) into a HIP graph and replayed (HLB_OPT_BATCH_GRAPH = 0: eager launches on a
 * stream-ordered workspace, with a synchronization of `stream` before return).
 *   probs: host array of `count` problems (count >= 0).  Output buffers must not overlap.
 * Results are bit-identical to calling hlb_cp_mm on each problem.
 */
hlb_status hlb_cp_mm_batch(const hlb_cpmm_problem *probs, int count, const uint64_t *primes,
                           int L, int form, void *stream);

/*
 * Synchronous check that every entry of a rows x cols residue matrix (row stride ld) is
 * < q (HLB_EINVAL on a stream under graph capture).  *first_bad (host) receives the row-major linear index (row*cols + col) of the first
 * offending entry, or -1.  Returns HLB_ERANGE if one exists, HLB_OK otherwise.
 */
hlb_status hlb_validate_residues(const uint64_t *X, int64_t rows, int64_t cols, int64_t ld,
                                 uint64_t q, int64_t *first_bad, void *stream);

/* Synchronous: *absmax (host) = max |P[i][j]| over an m x k signed matrix (row stride ld);
 * values equal to INT64_MIN report INT64_MAX.  HLB_EINVAL on a stream under graph capture. */
hlb_status hlb_plaintext_absmax(const int64_t *P, int64_t m, int64_t k, int64_t ld,
                                int64_t *absmax, void *stream);

/*
 * Plan the library would use (host only, no device work).
 *   Limb forms (Lemma le:strategy1): every partial sum of limb products must stay below 2^31
 *   in magnitude (INT8 digits, int32 accumulators) or 2^53 (FP64), so the plan fixes the
 *   limb counts and the number of K steps accumulated before a fold into a 64-bit residue.
 *   Multimodular form (Strategy 3): p_limbs = x_limbs = D, the number of moduli; their
 *   product is at least 4 k a floor(q/2) (a = p_absmax, or floor(q/2) for kind 0), and
 *   k <= 131071 keeps each modular product exact in int32.
 *   kind: 0 = Mod-PP-MM (P is a residue < q), 1 = CP-MM (|P| <= p_absmax).
 *   With HLB_FORM_AUTO the plan depends on k only; the product entry points also fall
 *   back from the multimodular to the digit form when m or n is below 256.
 */
typedef struct {
    int form;          /* HLB_FORM_INT8, HLB_FORM_INT8_CRT or HLB_FORM_FP64 */
    int p_limbs;       /* limbs (digits) of the left operand; multimodular: moduli */
    int x_limbs;       /* limbs (digits) of the right operand; multimodular: moduli */
    int shifts;        /* accumulators per output = p_limbs + x_limbs - 1 (limb forms) */
    int limb_bits;     /* bits per limb: 8 (INT8) or w (FP64) */
    int max_pairs;     /* largest number of limb products sharing one accumulator */
    int64_t k_chunk;   /* K elements accumulated before a fold (>= k means no fold) */
    double acc_bound_log2; /* log2 of the bound on |accumulator| used to size k_chunk */
} hlb_plan_desc;

hlb_status hlb_plan(int kind, int64_t k, uint64_t q_max, int64_t p_absmax, int form,
                    hlb_plan_desc *out);

/* Library options (process-wide).  Mainly for tests and measurement. */
typedef enum {
    HLB_OPT_FORCE_KCHUNK = 1, /* >0: cap the fold chunk at this many K elements (rounded to
                                 the kernel's K step); 0 restores the planned chunk */
    HLB_OPT_PROFILE = 2,      /* 1: bracket every kernel launch with HIP events */
    HLB_OPT_BATCH_GRAPH = 3,  /* 1 (default): capture/replay batches as HIP graphs; 0: eager */
    HLB_OPT_FORCE_CLASS = 4,  /* INT8 tile class: -1 (default) = tuned/heuristic choice,
                                 0 = 128 x 64 output tiles, 1 = 64 x 128 output tiles */
    HLB_OPT_F64_PLANES = 5,   /* FP64 form with one plaintext limb: 1 (default) = convert the
                                 operands into double planes (library workspace), then the
                                 direct-to-LDS GEMM; 0 = the register-staged kernel, which
                                 needs no workspace.  Results are identical. */
    HLB_OPT_CRT_WIDE = 6,     /* multimodular GEMM tile class: -1 (default) = per problem
                                 from the tuning table (256 x 384 where it has no entry);
                                 2 = 256 x 384 outputs, 1 = 256 x 256, 0 = 256 x 128 force a
                                 class for every call and batch problem; other values are
                                 refused with HLB_EINVAL.  Results are identical. */
    HLB_OPT_WS_CAP = 7,       /* > 0: refuse any single stream-ordered workspace allocation
                                 above this many bytes with HLB_ENOMEM, before any launch
                                 that would use it (a host-side way to exercise the
                                 out-of-memory paths); 0 (default): no cap.  Cached batch
                                 graphs allocate their own workspace and are not capped. */
    HLB_OPT_VALIDATE = 8      /* 1: hlb_mod_pp_mm, hlb_cp_mm and hlb_cp_mm_batch first check
                                 their inputs on the device -- every residue below its
                                 modulus (hlb_validate_residues), every |P| within p_absmax
                                 when one is given (hlb_plaintext_absmax) -- and return
                                 HLB_ERANGE before writing any output if one is not.  The
                                 checks synchronise the stream, so a capturing stream gets
                                 HLB_EINVAL.  hlb_cp_mm_noalloc and hlb_ccmm_pp_core do not
                                 check.  0 (default): no checks.  Starts at 1 when the
                                 environment holds HLB_VALIDATE=1. */
} hlb_option;

/*
 * Environment, read once per process:
 *   HLB_FORM=auto|fp64|int8|int8_crt  the form of every call that passes HLB_FORM_AUTO
 *                                      (hlb_plan included); explicit forms are kept.
 *   HLB_VALIDATE=1                     starts HLB_OPT_VALIDATE on.
 *   HLB_WS_CAP=bytes                   starts HLB_OPT_WS_CAP at that many bytes (a positive
 *                                      decimal integer; anything else leaves no cap).
 *   HLB_TUNE_CACHE=path                tuning table loaded before the first lookup
 *                                      (hlb_tune_load's format).
 */

hlb_status hlb_set_option(int option, int64_t value);

/*
 * Tile-class tuning table (host only).  The INT8 form has two workgroup tile classes; the
 * planner picks one per problem from this table, keyed by the ciphertext digit count and
 * the floor(log2) of the problem's rows m, columns n (of one output matrix) and depth k,
 * falling back to a padding-waste heuristic for keys it does not hold.  The autotuner
 * (paper_2503_16080_amd.autotune) measures both classes per key and fills the table.
 *   hlb_tune_set:   sets one entry (cls 0 or 1; cls -1 erases it).
 *   hlb_tune_load:  reads entries "x_digits log2m log2n log2k cls" (one per line, '#'
 *                   comments) from a text file; the library also loads the file named by
 *                   the environment variable HLB_TUNE_CACHE on first use.
 *   hlb_tune_class: the class the planner would use for a shape (-1 if none applies).
 */
hlb_status hlb_tune_set(int x_digits, int log2m, int log2n, int log2k, int cls);
hlb_status hlb_tune_load(const char *path);
int hlb_tune_class(int x_digits, int64_t m, int64_t n, int64_t k);

/*
 * The same table for the multimodular form (host only).  Its GEMM has three workgroup tile
 * classes: 0 = 256 x 128, 1 = 256 x 256, 2 = 256 x 384 outputs.  The planner picks one per
 * single call and per problem of a batch (a batch runs one persistent GEMM launch per class
 * present), keyed by the moduli count D and the floor(log2) of m, n (of one output matrix)
 * and k; class 2 where the table has no entry; HLB_OPT_CRT_WIDE >= 0 overrides it.
 *   hlb_tune_set_crt:   sets one entry (cls 0, 1 or 2; cls -1 erases it); HLB_EINVAL for
 *                       D outside 1..16, log2 fields outside 0..63 or another class.
 *   hlb_tune_load:      also reads entries "crt D log2m log2n log2k cls".
 *   hlb_tune_class_crt: the class the planner would use for a shape (-1 for invalid
 *                       arguments).
 */
hlb_status hlb_tune_set_crt(int moduli, int log2m, int log2n, int log2k, int cls);
int hlb_tune_class_crt(int moduli, int64_t m, int64_t n, int64_t k);

/*
 * Kernel timing collected while HLB_OPT_PROFILE is on (synchronous: waits for the
 * recorded events).  For kernel class `name`, *launches receives the number of launches and
 * *total_ms their summed durations measured between events recorded on each launch's stream.
 * Classes: multimodular form "crt_split" (residue splits of one call), "crt_gemm",
 * "crt_combine" (recombinations); its batch "crt_split_batch", "crt_gemm_batch",
 * "crt_combine_batch"; digit form "split_p", "split_x", "gemm_i8", "gemm_i8_trunc", its
 * batch "batch_i8"; FP64 form "prep_p", "prep_x", "gemm_f64", "gemm_f64_trunc".  Launches
 * inside a graph capture are not recorded.  Unknown names report zero.  Collected records
 * are cleared by hlb_profile_reset().
 */
hlb_status hlb_profile_read(const char *name, int64_t *launches, double *total_ms);
hlb_status hlb_profile_reset(void);

/* Frees the per-stream workspace blocks, pooled memory and cached batch graphs
 * (synchronises the device). */
hlb_status hlb_release(void);

/* ------------------------------------------------------------------------------------ */
/* Test-only helpers (not part of the product contract): CKKS coefficient encoding and a  */
/* matrix-form encryption/decryption, written from Section 2.2 and Eq mat_row_format.     */
/* ------------------------------------------------------------------------------------ */

/* out[i] = floor(delta * M[i] + 1/2) for `count` doubles (the paper's rounding). */
hlb_status hlb_test_encode(const double *M, int64_t count, double delta, int64_t *out,
                           void *stream);

/* B[l] = -(A[l] * S) + Menc (mod primes[l]) for l < L, where A: [L][k][n] residues,
 * S: n x n signed (int64, small), Menc: k x n signed (the encoded message plus error),
 * B: [L][k][n] output. */
hlb_status hlb_test_encrypt(int64_t k, int64_t n, const uint64_t *A, const int64_t *S,
                            const int64_t *Menc, const uint64_t *primes, int L, uint64_t *B,
                            void *stream);

/* D[l] = A[l] * S + B[l] (mod primes[l]); A, B: [L][rows][n], S: n x n signed, D output. */
hlb_status hlb_test_decrypt(int64_t rows, int64_t n, const uint64_t *A, const uint64_t *B,
                            const int64_t *S, const uint64_t *primes, int L, uint64_t *D,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HLB_H */
