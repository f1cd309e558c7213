"""Pins for the CPU oracle: checks against things other than the oracle itself.

Each test targets a plausible mistake in the oracle (dropped term, wrong index or stride,
transposed operand, sign error on negative plaintexts, accumulator overflow, wrong rounding
direction) using brute force on tiny inputs with Python integers, closed forms, algebraic
invariants, library routines on cases that reduce to them, and CKKS decryption identities.
"""
import itertools

import numpy as np
import pytest

import workloads as wl

PRIMES = [2, 3, 97, 65537, (1 << 31) - 1, wl.ntt_primes(50, 1)[0], wl.ntt_primes(52, 1)[0],
          (1 << 61) - 1]


def _brute(q, P, X):
    m, k = len(P), len(P[0])
    n = len(X[0])
    return [[sum(int(P[i][l]) * int(X[l][j]) for l in range(k)) % q for j in range(n)]
            for i in range(m)]


def _edge_values(q):
    vals = {0, 1, q - 1, q - 2, (q - 1) // 2, (q + 1) // 2}
    return sorted(v for v in vals if 0 <= v < q)


@pytest.mark.parametrize("q", PRIMES)
def test_brute_force_tiny(orc, q):
    g = np.random.default_rng(q % 1000 + 7)
    edges = _edge_values(q)
    for (m, k, n) in [(1, 1, 1), (2, 3, 4), (5, 1, 3), (3, 7, 2), (9, 9, 9), (4, 8, 1)]:
        P = g.integers(0, q, size=(m, k), dtype=np.uint64)
        X = g.integers(0, q, size=(k, n), dtype=np.uint64)
        # sprinkle extremal residues
        P.flat[g.integers(0, P.size)] = edges[g.integers(0, len(edges))]
        X.flat[g.integers(0, X.size)] = edges[g.integers(0, len(edges))]
        got = orc.mod_pp_mm(q, P, X)
        assert got.tolist() == _brute(q, P.tolist(), X.tolist())


@pytest.mark.parametrize("q", PRIMES[1:])
def test_all_q_minus_one_closed_form(orc, q):
    # (q-1)^2 = 1 mod q, so every output is k mod q.
    for (m, k, n) in [(3, 1, 2), (4, 17, 5), (2, 300, 3)]:
        P = np.full((m, k), q - 1, dtype=np.uint64)
        X = np.full((k, n), q - 1, dtype=np.uint64)
        assert (orc.mod_pp_mm(q, P, X) == k % q).all()


def test_accumulator_fold_large_k(orc):
    # 2^61-1 allows only a few dozen (q-1)^2 terms per 128-bit accumulator before folding;
    # a 52-bit prime allows ~2^24.  Both must still give k mod q.
    for q, k in [((1 << 61) - 1, 1000), ((1 << 61) - 1, 129), (wl.ntt_primes(52, 1)[0], (1 << 24) + 3)]:
        P = np.full((1, k), q - 1, dtype=np.uint64)
        X = np.full((k, 1), q - 1, dtype=np.uint64)
        assert int(orc.mod_pp_mm(q, P, X)[0, 0]) == k % q


@pytest.mark.parametrize("q", PRIMES[2:])
def test_identity_and_diagonal(orc, q):
    g = np.random.default_rng(5)
    P = g.integers(0, q, size=(6, 6), dtype=np.uint64)
    I = np.eye(6, dtype=np.uint64)
    assert (orc.mod_pp_mm(q, P, I) == P).all()
    assert (orc.mod_pp_mm(q, I, P) == P).all()
    c = g.integers(0, q, size=6)
    D = np.diag(c).astype(np.uint64)
    X = g.integers(0, q, size=(6, 4), dtype=np.uint64)
    want = [[int(c[i]) * int(X[i, j]) % q for j in range(4)] for i in range(6)]
    assert orc.mod_pp_mm(q, D, X).tolist() == want


@pytest.mark.parametrize("q", PRIMES[2:])
def test_ones_gives_column_sums(orc, q):
    g = np.random.default_rng(11)
    X = g.integers(0, q, size=(13, 5), dtype=np.uint64)
    ones = np.ones((3, 13), dtype=np.uint64)
    col = [sum(int(v) for v in X[:, j]) % q for j in range(5)]
    got = orc.mod_pp_mm(q, ones, X)
    assert all(got[i].tolist() == col for i in range(3))


@pytest.mark.parametrize("q", PRIMES[2:])
def test_single_entries_outer_product(orc, q):
    # P has one nonzero at (a, b), X one nonzero at (b, c): C is zero except C[a, c].
    a, b, c = 2, 3, 1
    alpha, beta = q - 3, q // 2 + 1
    P = np.zeros((4, 5), dtype=np.uint64)
    X = np.zeros((5, 3), dtype=np.uint64)
    P[a, b] = alpha
    X[b, c] = beta
    C = orc.mod_pp_mm(q, P, X)
    want = np.zeros((4, 3), dtype=object)
    want[a, c] = alpha * beta % q
    assert C.astype(object).tolist() == want.tolist()
    # a mismatched inner index gives zero: catches a transposed operand
    X2 = np.zeros((5, 3), dtype=np.uint64)
    X2[b + 1, c] = beta
    assert (orc.mod_pp_mm(q, P, X2) == 0).all()


@pytest.mark.parametrize("q", PRIMES[3:])
def test_linearity_and_associativity(orc, q):
    g = np.random.default_rng(q % 997)
    P1 = g.integers(0, q, size=(7, 11), dtype=np.uint64)
    P2 = g.integers(0, q, size=(7, 11), dtype=np.uint64)
    X = g.integers(0, q, size=(11, 5), dtype=np.uint64)
    Y = g.integers(0, q, size=(5, 3), dtype=np.uint64)
    Psum = ((P1.astype(object) + P2.astype(object)) % q).astype(np.uint64)
    lhs = orc.mod_pp_mm(q, Psum, X).astype(object)
    rhs = (orc.mod_pp_mm(q, P1, X).astype(object) + orc.mod_pp_mm(q, P2, X).astype(object)) % q
    assert lhs.tolist() == rhs.tolist()
    # (P X) Y == P (X Y) mod q on non-square shapes (fails for a transposed operand)
    left = orc.mod_pp_mm(q, orc.mod_pp_mm(q, P1, X), Y)
    right = orc.mod_pp_mm(q, P1, orc.mod_pp_mm(q, X, Y))
    assert (left == right).all()


def test_small_values_match_integer_matmul(orc):
    # When the exact integer product is below q, Mod-PP-MM is the plain integer matmul.
    q = wl.ntt_primes(50, 1)[0]
    g = np.random.default_rng(3)
    P = g.integers(0, 1000, size=(23, 41))
    X = g.integers(0, 1000, size=(41, 19))
    assert (orc.mod_pp_mm(q, P, X).astype(np.int64) == P @ X).all()


def test_rows_subset_matches_full(orc):
    q = wl.ntt_primes(50, 1, skip=2)[0]
    g = np.random.default_rng(4)
    P = g.integers(0, q, size=(17, 9), dtype=np.uint64)
    X = g.integers(0, q, size=(9, 6), dtype=np.uint64)
    full = orc.mod_pp_mm(q, P, X)
    rows = [0, 5, 16, 7]
    part = orc.mod_pp_mm(q, P, X, rows=rows)
    assert (part[rows] == full[rows]).all()
    others = [r for r in range(17) if r not in rows]
    assert (part[others] == 0).all()


def test_residues_of_signed_are_floor_mod(orc):
    for q in [3, 97, wl.ntt_primes(50, 1)[0], (1 << 61) - 1]:
        vals = np.array([0, 1, -1, 5, -5, q - 1, -(q - 1), -q, q, -(1 << 62), -(1 << 63),
                         (1 << 63) - 1, -12345678901], dtype=np.int64)
        got = orc.residues_of_signed(vals, q).tolist()
        assert got == [int(v) % q for v in vals.tolist()]  # Python % is floor-mod


def test_cp_mm_negative_plaintext(orc):
    primes = wl.ntt_primes(50, 3)
    g = np.random.default_rng(8)
    P = g.integers(-(1 << 20), (1 << 20) + 1, size=(6, 10))
    A = np.stack([g.integers(0, 50, size=(10, 4)) for _ in primes]).astype(np.uint64)
    B = np.stack([g.integers(0, 50, size=(10, 5)) for _ in primes]).astype(np.uint64)
    PA, PB = orc.cp_mm(P, A, B, primes)
    for i, q in enumerate(primes):
        # exact integer products (|.| < 2^30) reduced with Python's floor-mod
        assert PA[i].astype(object).tolist() == ((P @ A[i].astype(np.int64)).astype(object) % q).tolist()
        assert PB[i].astype(object).tolist() == ((P @ B[i].astype(np.int64)).astype(object) % q).tolist()


def test_cp_mm_full_residues_brute(orc):
    primes = wl.ntt_primes(45, 2)
    g = np.random.default_rng(9)
    P = g.integers(-(1 << 20), (1 << 20) + 1, size=(3, 5))
    A = np.stack([g.integers(0, q, size=(5, 4), dtype=np.uint64) for q in primes])
    B = np.stack([g.integers(0, q, size=(5, 2), dtype=np.uint64) for q in primes])
    PA, PB = orc.cp_mm(P, A, B, primes)
    for i, q in enumerate(primes):
        Pq = [[int(v) % q for v in row] for row in P.tolist()]
        assert PA[i].tolist() == _brute(q, Pq, A[i].tolist())
        assert PB[i].tolist() == _brute(q, Pq, B[i].tolist())


def test_matvec_matches_brute_and_product(orc):
    q = wl.ntt_primes(52, 1)[0]
    g = np.random.default_rng(10)
    M = g.integers(0, q, size=(9, 14), dtype=np.uint64)
    v = g.integers(0, q, size=14, dtype=np.uint64)
    got = orc.matvec_mod(q, M, v)
    assert got.tolist() == [r[0] for r in _brute(q, M.tolist(), [[int(x)] for x in v])]


def test_freivalds_detects_planted_error(orc):
    # A product with one wrong entry fails P(Xr) = Cr for a random r (prob. error <= 1/q).
    q = wl.ntt_primes(50, 1)[0]
    g = np.random.default_rng(12)
    P = g.integers(0, q, size=(20, 30), dtype=np.uint64)
    X = g.integers(0, q, size=(30, 25), dtype=np.uint64)
    C = orc.mod_pp_mm(q, P, X)
    r = g.integers(0, q, size=25, dtype=np.uint64)
    lhs = orc.matvec_mod(q, P, orc.matvec_mod(q, X, r))
    assert (lhs == orc.matvec_mod(q, C, r)).all()
    C[7, 11] = (int(C[7, 11]) + 1) % q
    assert not (lhs == orc.matvec_mod(q, C, r)).all()


def test_precondition_rejects_non_residues(orc):
    q = 97
    P = np.array([[1, 97]], dtype=np.uint64)
    X = np.array([[1], [1]], dtype=np.uint64)
    with pytest.raises(ValueError):
        orc.mod_pp_mm(q, P, X)


# ------------------------------- CKKS helpers ------------------------------------------

def test_round_half_up_ties(orc):
    x = np.array([2.5, -2.5, 0.5, -0.5, 1.49999, -1.5, -2.7, 3.0, -0.0])
    assert orc.round_half_up(x).tolist() == [3, -2, 1, 0, 1, -1, -3, 3, 0]


def test_crt_lift_small_primes(orc):
    primes = [3, 5, 7]   # Q = 105, centred range (-52, 52]
    for v in [-52 + 1, -17, -1, 0, 1, 17, 52]:
        D = np.array([[v % 3], [v % 5], [v % 7]], dtype=np.uint64).reshape(3, 1)
        assert orc.crt_lift_centered(D, primes)[0] == v


def test_precision_metric(orc):
    M = np.array([1.0, -0.5, 0.25])
    Mt = M + np.array([0.0, 2.0 ** -10, -(2.0 ** -12)])
    assert orc.precision_bits(M, Mt) == pytest.approx(10.0)


def test_encrypt_decrypt_identity(orc):
    # A S + B = encode(M) + E (mod q_i) exactly, for every prime.
    d = wl.ckks_draws(seed=21, m=4, k=12, n=10, bits=50, L=3)
    delta = 2.0 ** d.delta_bits
    Menc = orc.encode(d.M, delta)
    B = orc.encrypt(d.A, d.S, Menc, d.E, d.primes)
    D = orc.decrypt(d.A, B, d.S, d.primes)
    for i, q in enumerate(d.primes):
        assert D[i].astype(object).tolist() == ((Menc + d.E).astype(object) % q).tolist()
    lifted = orc.crt_lift_centered(D, d.primes)
    assert lifted.astype(np.int64).tolist() == (Menc + d.E).tolist()


def test_cp_mm_then_decrypt_is_plaintext_product(orc):
    # Left-multiplying the ciphertext by P keeps the decryption identity (Eq LZoutput in
    # row form):  (P A) S + P B = P (encode(M) + E)  (mod each q_i), checked exactly after
    # CRT lifting with Python integers, and decoded within the noise bound.
    d = wl.ckks_draws(seed=22, m=6, k=16, n=9, bits=50, L=3)
    delta = 2.0 ** d.delta_bits
    Menc = orc.encode(d.M, delta)
    B = orc.encrypt(d.A, d.S, Menc, d.E, d.primes)
    P = orc.round_half_up(d.U * 2.0 ** d.p_scale_bits)
    PA, PB = orc.cp_mm(P, d.A, B, d.primes)
    D = orc.decrypt(PA, PB, d.S, d.primes)
    lifted = orc.crt_lift_centered(D, d.primes)
    exact = P.astype(object) @ (Menc + d.E).astype(object)
    assert lifted.tolist() == exact.tolist()
    # decode: D / (Delta * 2^20) approximates Pq M / 2^20 with error <= k |P| (|E| + 1/2) / (Delta 2^20)
    got = orc.decode(lifted, delta * 2.0 ** d.p_scale_bits)
    ref = (P.astype(np.float64) @ d.M) / 2.0 ** d.p_scale_bits
    bound = d.M.shape[0] * np.abs(P).max() * (np.abs(d.E).max() + 0.5) / (delta * 2.0 ** d.p_scale_bits)
    assert np.abs(got - ref).max() <= bound


# ------------------------------- input generators -------------------------------------

def test_prime_generation():
    assert wl.is_prime((1 << 61) - 1)
    assert wl.is_prime((1 << 64) - 59)
    assert wl.is_prime(0xFFFFFFFF00000001)
    for c in [1, 561, 3215031751, 25326001, (1 << 61) + 1, 341550071728321]:
        assert not wl.is_prime(c)
    ps = wl.ntt_primes(50, 4)
    assert ps == sorted(ps, reverse=True) and len(set(ps)) == 4
    for q in ps:
        assert q < (1 << 50) and q > (1 << 49) and q % (1 << 17) == 1 and wl.is_prime(q)
    # nothing skipped between consecutive picks
    step = 1 << 17
    for a, b in itertools.pairwise(ps):
        assert not any(wl.is_prime(x) for x in range(b + step, a, step))
    assert wl.ntt_primes(50, 2, skip=1) == ps[1:3]


def test_golden_regression_fixture(orc):
    # Stored values (written by tests/golden/make_golden.py from the oracle) must not drift;
    # their corner entries are re-derived here by Python-integer brute force.
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_regression.json")
    with open(path) as f:
        cases = json.load(f)["cases"]
    h = lambda a: hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()
    for c in cases:
        if c["kind"] == "mod_pp_mm":
            g = wl.rng(c["seed"])
            q = c["q"]
            P = wl.uniform_residues(g, (c["m"], c["k"]), q)
            X = wl.uniform_residues(g, (c["k"], c["n"]), q)
            assert h(orc.mod_pp_mm(q, P, X)) == c["sha256"]
            assert sum(int(P[0, l]) * int(X[l, 0]) for l in range(c["k"])) % q == c["corner"][0]
            assert sum(int(P[-1, l]) * int(X[l, -1]) for l in range(c["k"])) % q == c["corner"][1]
        else:
            w = wl.cpmm_uniform(c["seed"], c["m"], c["k"], c["n"], c["bits"], c["L"])
            assert w.primes == c["primes"]
            PA, PB = orc.cp_mm(w.P, w.A, w.B, w.primes)
            assert h(PA) == c["sha256_PA"] and h(PB) == c["sha256_PB"]
            q0, qL = w.primes[0], w.primes[-1]
            assert sum(int(w.P[0, l]) * int(w.A[0, l, 0]) for l in range(c["k"])) % q0 == c["corner"][0]
            assert sum(int(w.P[-1, l]) * int(w.B[-1, l, -1]) for l in range(c["k"])) % qL == c["corner"][1]


def test_rescale_definition_pins(orc):
    # (1) brute force with exact fractions, ties rounded upward; (2) x = q y + e recovers
    # y + round(e / q); (3) the result does not depend on the representative of x mod Q.
    from fractions import Fraction
    import math
    primes = [97, 101, 103]
    Q = 97 * 101 * 103
    q = 103
    xs = [0, 1, 51, 52, 103, 154, 155, 5000, Q - 1, Q // 2, Q // 2 + 1, 206 + 51, 206 + 52]
    X = np.array([[x % p for x in xs] for p in primes], dtype=np.uint64)
    got = orc.rescale(X, primes)
    for i, x in enumerate(xs):
        xc = x - Q if x > Q // 2 else x          # the centred representative is what is lifted
        want = math.floor(Fraction(xc, q) + Fraction(1, 2))
        assert [int(got[l, i]) for l in range(2)] == [want % 97, want % 101]
    primes = wl.ntt_primes(50, 3)
    g = np.random.default_rng(17)
    q = primes[-1]
    y = g.integers(-(1 << 40), 1 << 40, size=50)
    e = g.integers(-(q // 2) + 1, q // 2, size=50)
    x = [int(a) * q + int(b) for a, b in zip(y, e)]
    X = np.array([[v % p for v in x] for p in primes], dtype=np.uint64)
    got = orc.rescale(X, primes)
    for l in range(2):
        assert got[l].tolist() == [int(a) % primes[l] for a in y]
    # ties: e = q/2 rounds up (q odd: e = (q+1)/2 up, (q-1)/2 down)
    x = [5 * q + (q + 1) // 2, 5 * q + (q - 1) // 2]
    X = np.array([[v % p for v in x] for p in primes], dtype=np.uint64)
    assert orc.rescale(X, primes)[0].tolist() == [6, 5]


def test_ccmm_core_composes_definitions(orc):
    primes = wl.ntt_primes(50, 2)
    g = np.random.default_rng(18)
    A, B = (np.stack([g.integers(0, q, size=(4, 6), dtype=np.uint64) for q in primes]) for _ in range(2))
    At, Bt = (np.stack([g.integers(0, q, size=(6, 5), dtype=np.uint64) for q in primes]) for _ in range(2))
    C = orc.ccmm_pp_core(A, B, At, Bt, primes)
    for l, q in enumerate(primes):
        top = np.concatenate([A[l], B[l]]).tolist()
        right = np.concatenate([At[l], Bt[l]], axis=1).tolist()
        full = _brute(q, top, right)   # [A; B] * [At Bt] as one product
        assert C[0][l].tolist() == [r[:5] for r in full[:4]]
        assert C[1][l].tolist() == [r[5:] for r in full[:4]]
        assert C[2][l].tolist() == [r[:5] for r in full[4:]]
        assert C[3][l].tolist() == [r[5:] for r in full[4:]]
