"""Pins for the oracle's Strategy 2 (truncation) functions, Section 6.1.

Each test checks the approximate products against something other than themselves: the
exact Mod-PP-MM where truncation must lose nothing, Python-integer brute force over the
digits, the error bounds the method guarantees, and inputs built so that a missing step
(no centring, wrong digit range, wrong shift set) changes the result.
"""
import numpy as np
import pytest

import workloads as wl

Q50 = wl.ntt_primes(50, 1)[0]


def _centred_diff(a, b, q):
    d = (a.astype(object) - b.astype(object)) % q
    return np.where(d > q // 2, d - q, d)


def _pairs(s, dp, dx):
    return sum(1 for i in range(dp) if 0 <= s - i < dx)


def test_balanced_digits_round_trip_and_range(orc):
    g = np.random.default_rng(1)
    for D in (1, 3, 6, 7):
        cap = sum(127 * 256 ** j for j in range(D))          # largest value D digits hold
        low = -sum(128 * 256 ** j for j in range(D))          # smallest
        v = np.concatenate([g.integers(low, cap + 1, size=500), [0, 1, -1, cap, low, 127, -128],
                            [128, -129] if D > 1 else []]).astype(np.int64)
        d = orc.balanced_digits(v, D)
        assert all(int(x.min()) >= -128 and int(x.max()) <= 127 for x in d)
        back = sum(x.astype(object) * 256 ** j for j, x in enumerate(d))
        assert back.tolist() == v.tolist()
        with pytest.raises(ValueError):
            orc.balanced_digits(np.array([cap + 1]), D)
        with pytest.raises(ValueError):
            orc.balanced_digits(np.array([low - 1]), D)
    # 50-bit residues need exactly 7 digits (q - 1 > capacity of 6)
    assert orc.balanced_digits(np.array([Q50 - 1]), 7)
    with pytest.raises(ValueError):
        orc.balanced_digits(np.array([Q50 - 1]), 6)


def test_drop_zero_is_the_exact_product(orc):
    g = wl.rng(3)
    P = wl.plaintext_matrix(g, 9, 70)
    X = wl.uniform_residues(g, (70, 11), Q50)
    exact = orc.mod_pp_mm(Q50, orc.residues_of_signed(P, Q50), X)
    assert np.array_equal(orc.mod_pp_mm_drop_i8(Q50, P, X, 0, 3, 7), exact)


@pytest.mark.parametrize("drop", [1, 2, 3])
def test_drop_matches_digit_brute_force(orc, drop):
    # Python-integer brute force: per output, the double sum over K and over the kept digit
    # pairs, digits from plain divmod (not from the oracle's digit routine)
    def digits(v, D):
        out = []
        for _ in range(D):
            d = (v + 128) % 256 - 128
            out.append(d)
            v = (v - d) // 256
        assert v == 0
        return out

    g = wl.rng(10 + drop)
    m, k, n = 3, 5, 4
    P = wl.plaintext_matrix(g, m, k)
    X = wl.uniform_residues(g, (k, n), Q50)
    got = orc.mod_pp_mm_drop_i8(Q50, P, X, drop, 3, 7)
    for i in range(m):
        for j in range(n):
            t = 0
            for l in range(k):
                pd, xd = digits(int(P[i, l]), 3), digits(int(X[l, j]), 7)
                t += sum(pd[a] * xd[b] * 256 ** (a + b) for a in range(3) for b in range(7) if a + b >= drop)
            assert int(got[i, j]) == t % Q50


@pytest.mark.parametrize("dx,bits", [(7, 50), (6, 45)])
def test_drop_error_within_bound_and_nonzero(orc, dx, bits):
    q = wl.ntt_primes(bits, 1)[0]
    g = wl.rng(20 + dx)
    k = 300
    P = wl.plaintext_matrix(g, 12, k)
    X = wl.uniform_residues(g, (k, 13), q)
    exact = orc.mod_pp_mm(q, orc.residues_of_signed(P, q), X)
    for drop in (1, 2, 3):
        got = orc.mod_pp_mm_drop_i8(q, P, X, drop, 3, dx)
        err = np.abs(_centred_diff(got, exact, q)).max()
        bound = k * 2 ** 14 * sum(_pairs(s, 3, dx) * 256 ** s for s in range(drop))
        assert 0 < err <= bound
        # the dropped part is an exact integer: exact - got equals the low-shift sum
        Pd = orc.balanced_digits(P, 3)
        Xd = orc.balanced_digits(X.astype(np.int64), dx)
        low = sum((Pd[a] @ Xd[b]).astype(object) * 256 ** (a + b)
                  for a in range(3) for b in range(dx) if a + b < drop)
        assert np.array_equal(_centred_diff(exact, got, q), low)


def test_fp64_trunc_exact_when_partial_sums_stay_below_2_53(orc):
    # k |P| q/2 < 2^53: every rounding is exact, so Strategy 2 returns the exact product
    g = wl.rng(30)
    for q in (97, 65537, (1 << 31) - 1):
        k = 64
        P = g.integers(-(1 << 15), 1 << 15, size=(7, k))
        X = g.integers(0, q, size=(k, 9), dtype=np.uint64)
        assert k * (1 << 15) * (q // 2) < 2 ** 53
        assert np.array_equal(orc.mod_pp_mm_trunc_fp64(q, P, X),
                              orc.mod_pp_mm(q, orc.residues_of_signed(P, q), X))


def test_fp64_trunc_centres_the_residues(orc):
    # X = q - 1 is -1 in centred form: P X = -(row sums of P), exact in doubles; without the
    # centring the products P (q - 1) ~ 2^70 would round and the result would be wrong
    q = Q50
    g = wl.rng(31)
    k = 4096
    P = wl.plaintext_matrix(g, 5, k)
    X = np.full((k, 3), q - 1, dtype=np.uint64)
    want = orc.mod_pp_mm(q, orc.residues_of_signed(P, q), X)
    assert np.array_equal(orc.mod_pp_mm_trunc_fp64(q, P, X), want)
    # entries just above q/2 are negative, just below stay positive
    X = np.array([[(q + 1) // 2, (q - 1) // 2]], dtype=np.uint64)
    c = orc.centred(X, q)
    assert c.tolist() == [[(q + 1) // 2 - q, (q - 1) // 2]]


def test_fp64_trunc_error_within_worst_case_bound(orc):
    q = Q50
    g = wl.rng(32)
    k = 1024
    P = wl.plaintext_matrix(g, 16, k)
    X = wl.uniform_residues(g, (k, 16), q)
    exact = orc.mod_pp_mm(q, orc.residues_of_signed(P, q), X)
    got = orc.mod_pp_mm_trunc_fp64(q, P, X)
    err = np.abs(_centred_diff(got, exact, q)).astype(float)
    absum = np.abs(P).astype(float) @ np.abs(orc.centred(X, q)).astype(float)
    bound = (k + 2) * 2.0 ** -52 * absum * (1 + 1e-9)
    assert np.all(err <= bound)
    assert err.max() > 0          # the method is approximate at this size
    # and within the paper's heuristic size 2^-50 k |P| |X| for these uniform inputs
    assert err.max() <= 2.0 ** -50 * k * np.abs(P).max() * (q / 2)
