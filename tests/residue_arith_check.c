/* residue_arith_check.c -- CPU check of the integer constructions the multimodular split
 * uses on the GPU, against residues computed with plain integer division.
 *
 *  residue(s, p), |s| < 2^52: t = nearest integer to s / p, read from the low word of the
 *    double fma(s, 1/p, 1.5 2^52); w = (t mod 2^24) (2^24 - p) + s (mod 2^32); the low byte
 *    of w must be the balanced residue of s (for p = 256: congruent modulo 256), and for
 *    p < 256 the low 24 bits of w read as a signed number must be that residue.
 *  small(x, p), |x| < 2^23: the same with the float fma(x, 1/p, 1.5 2^23), whose low 24 bits
 *    hold 2^22 + t; the low byte of w must again be the balanced residue.
 *
 * Usage: residue_arith_check <random values per modulus>.  Prints "ok <checks>" or the first
 * mismatch, and exits non-zero on a mismatch. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static const int kMods[16] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191};

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static uint64_t next(void) { /* splitmix64 */
    uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static int balanced(int64_t s, int p) {
    int64_t r = s % p;
    if (r < 0) r += p;
    if (r > (p - 1) / 2) r -= p;
    return (int)r;
}

static uint32_t residue_word(int64_t s, int p) {
    if (p == 256) return (uint32_t)s;
    const double sd = fma((double)(int32_t)(s >> 32), 4294967296.0, (double)(uint32_t)s);
    const double td = fma(sd, 1.0 / (double)p, 6755399441055744.0);
    uint64_t bits;
    memcpy(&bits, &td, 8);
    return ((uint32_t)bits & 0xffffffu) * ((1u << 24) - (uint32_t)p) + (uint32_t)s;
}

static uint32_t small_word(int32_t x, int p) {
    const float tf = fmaf((float)x, 1.0f / (float)p, 12582912.0f);
    uint32_t bits;
    memcpy(&bits, &tf, 4);
    return (bits & 0xffffffu) * ((1u << 24) - (uint32_t)p) + (uint32_t)x;
}

static long checks = 0;

static int same(int want, uint32_t w, int p) {
    const int got = (int8_t)(uint8_t)(w & 0xffu);
    return p == 256 ? ((want - got) % 256 == 0) : want == got;
}

static void check_value(int64_t s, int p) {
    const int64_t lim = ((int64_t)1 << 52) - 1;
    if (s > lim || s < -lim) return;
    ++checks;
    const uint32_t w = residue_word(s, p);
    const int want = balanced(s, p);
    if (!same(want, w, p) || (p < 256 && ((int32_t)(w << 8) >> 8) != want)) {
        printf("residue mismatch p=%d s=%lld want=%d word=%08x\n", p, (long long)s, want, w);
        exit(1);
    }
}

int main(int argc, char **argv) {
    const long n = argc > 1 ? atol(argv[1]) : 100000;
    const int64_t lim = ((int64_t)1 << 52) - 1;
    for (int i = 0; i < 16; ++i) {
        const int p = kMods[i];
        for (long j = 0; j < n; ++j) { /* magnitudes spread over every bit length */
            int64_t s = (int64_t)(next() & ((1ull << (1 + next() % 52)) - 1));
            check_value(next() & 1 ? -s : s, p);
        }
        for (long j = 0; j < n / 16; ++j) { /* around half-integer quotients at the top */
            int64_t t = (int64_t)(next() % (uint64_t)(lim / p));
            if (next() & 1) t = -t;
            for (int d = -(p / 2) - 1; d <= p / 2 + 1; ++d)
                if (d < -(p / 2) + 2 || d > p / 2 - 2) check_value(t * p + d, p);
        }
        for (int64_t d = 0; d < 4096; ++d) { check_value(lim - d, p); check_value(-lim + d, p); check_value(d - 2048, p); }
        for (int32_t x = -(1 << 16); x <= (1 << 16); ++x) { /* the scaled residues: |x| < 2^15 */
            ++checks;
            if (!same(balanced(x, p), small_word(x, p), p)) {
                printf("small mismatch p=%d x=%d\n", p, x);
                return 1;
            }
        }
    }
    printf("ok %ld\n", checks);
    return 0;
}
