/*
 * oracle.c -- CPU oracle for modular plaintext matrix products (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the slow, obviously-correct reference that the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant with the GPU library.
 *
 * What it computes is the plain definition of Mod-PP-MM (Section 5, the notation
 * Mod-PP-MM_{q; d1,d2,d3}: the product of two integer matrices reduced modulo q), written
 * out as a schoolbook dot product per output with exact 128-bit accumulation and one final
 * reduction into the canonical range [0, q).  The paper reaches the same integer result by
 * splitting the operands into small limbs, multiplying the limbs exactly in floating point
 * and recombining over the integers before reducing modulo q (Section 6.1, Strategy 1,
 * Lemma le:strategy1); since that route is exact, its result IS this definition.
 *
 * CP-MM (Algorithm alg:pcmm, step 1; Theorem th:pcmm-shs) is two Mod-PP-MMs per modulus;
 * the Python wrapper composes it from the functions here.
 *
 * Exactness: operands are canonical residues < q < 2^63, so each product is < 2^126.  The
 * 128-bit accumulator is folded back below q after every `fold` terms, where `fold` is the
 * largest count with q + fold*(q-1)^2 < 2^128 (capped at 2^30), so it never wraps.
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of products that can be added to an accumulator < q without passing 2^128. */
static int64_t oracle_fold_interval(uint64_t q) {
    const u128 top = ~(u128)0;
    const u128 sq = (u128)(q - 1) * (u128)(q - 1);
    if (sq == 0) return (int64_t)1 << 30;
    u128 t = (top - q) / sq;
    if (t > ((u128)1 << 30)) t = (u128)1 << 30;
    return (int64_t)t;
}

/* One output of the definition: (sum_l p[l*sp] * x[l*sx]) mod q.  Sets *bad if an
 * operand is not a canonical residue (precondition of the caller). */
static uint64_t oracle_dot_mod(uint64_t q, int64_t k, const uint64_t *p, int64_t sp,
                               const uint64_t *x, int64_t sx, int64_t fold, int *bad) {
    u128 acc = 0;
    int64_t since_fold = 0;
    for (int64_t l = 0; l < k; ++l) {
        const uint64_t a = p[l * sp];
        const uint64_t b = x[l * sx];
        if (a >= q || b >= q) *bad = 1;
        acc += (u128)a * (u128)b;
        if (++since_fold == fold) {
            acc %= q;
            since_fold = 0;
        }
    }
    return (uint64_t)(acc % q);
}

/*
 * C[i][j] = (sum_l P[i][l] * X[l][j]) mod q for the rows i listed in rows[0..nrows).
 * P: residues with row stride ldp; X: k x n residues with row stride ldx.
 * C[i*ldc + j] is written for listed rows only.
 * Returns 0 on success, 1 if some input is >= q (precondition violated), 2 on bad args.
 */
int oracle_mod_pp_mm_rows(uint64_t q, int64_t nrows, const int64_t *rows, int64_t k, int64_t n,
                          const uint64_t *P, int64_t ldp, const uint64_t *X, int64_t ldx,
                          uint64_t *C, int64_t ldc) {
    if (q < 2 || k < 0 || n < 0 || nrows < 0) return 2;
    const int64_t fold = oracle_fold_interval(q);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad) collapse(2)
    for (int64_t r = 0; r < nrows; ++r) {
        for (int64_t j = 0; j < n; ++j) {
            const int64_t i = rows[r];
            int b = 0;
            C[i * ldc + j] = oracle_dot_mod(q, k, P + i * ldp, 1, X + j, ldx, fold, &b);
            bad |= b;
        }
    }
    return bad ? 1 : 0;
}

/* The full Mod-PP-MM: every row of C = P * X mod q (P: m x k, X: k x n). */
int oracle_mod_pp_mm(uint64_t q, int64_t m, int64_t k, int64_t n, const uint64_t *P,
                     int64_t ldp, const uint64_t *X, int64_t ldx, uint64_t *C, int64_t ldc) {
    if (q < 2 || m < 0 || k < 0 || n < 0) return 2;
    const int64_t fold = oracle_fold_interval(q);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad) collapse(2)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            int b = 0;
            C[i * ldc + j] = oracle_dot_mod(q, k, P + i * ldp, 1, X + j, ldx, fold, &b);
            bad |= b;
        }
    }
    return bad ? 1 : 0;
}

/* Matrix-vector product mod q: out[i] = (sum_l M[i][l] * v[l]) mod q (Freivalds checks). */
int oracle_matvec_mod(uint64_t q, int64_t rows, int64_t cols, const uint64_t *M, int64_t ldm,
                      const uint64_t *v, uint64_t *out) {
    if (q < 2 || rows < 0 || cols < 0) return 2;
    const int64_t fold = oracle_fold_interval(q);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < rows; ++i) {
        int b = 0;
        out[i] = oracle_dot_mod(q, cols, M + i * ldm, 1, v, 1, fold, &b);
        bad |= b;
    }
    return bad ? 1 : 0;
}

/* Canonical residue of a signed integer: the representative of v modulo q in [0, q). */
static uint64_t oracle_residue_of_signed(int64_t v, uint64_t q) {
    if (v >= 0) return (uint64_t)v % q;
    const uint64_t mag = (uint64_t)(-(v + 1)) + 1u; /* |v| without overflow at INT64_MIN */
    const uint64_t r = mag % q;
    return r == 0 ? 0 : q - r;
}

/* out[i] = v[i] mod q in [0, q), for a signed plaintext matrix stored densely. */
void oracle_residues_of_signed(uint64_t q, int64_t count, const int64_t *v, uint64_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) out[i] = oracle_residue_of_signed(v[i], q);
}
