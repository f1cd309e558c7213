"""GPU parity at the remaining benchmark configurations, in the launch configuration the
benchmark times:

* the large CP-MM: d = 16384 over 2 primes of 50 bits (Table tab:pcmm's largest size), in the
  multimodular and digit INT8 forms;
* the batch: 64 CP-MMs of uneven shapes (m, d log-uniform, n = d) over 4 primes of 45 bits,
  one batch call in each batch form (Theorem th:pcmm-shs applied to every problem);
* the end-to-end CKKS check in the multimodular form at d = 4096 and at the headline size
  d = 8192 over 3 primes, and at d = 16384 over 2 primes: a real encryption (Eq
  mat_row_format), the product, decryption (Section 2.2 Dec), the CRT lift and decoding,
  within the noise bound.

Every output matrix is checked by Freivalds' test against the oracle (P (X r) = C r mod q for
random r; a wrong matrix passes one vector with probability <= 1/q), and sampled rows (first,
last, the 256-row tile edge, one inside) are compared with the oracle's rows element by
element.  Inputs are drawn on the device by the seeded generators of ``workloads`` and copied to
the host for the oracle; nothing the oracle sees comes from the library."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_16080_amd as hlb
import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _host(t):
    """A device int64 tensor as a host uint64 array (bit-identical for residues)."""
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 else a


def _rows(m):
    return sorted({0, min(1, m - 1), min(255, m - 1), min(256, m - 1), m // 2 + 3 if m > 8 else m - 1, m - 1})


class _Expect:
    """Oracle expectations of one CP-MM: its sampled rows and, per Freivalds vector, the left
    side P (X r) mod q of every output matrix."""

    def __init__(self, P, A, B, primes, rows, vectors, seed):
        self.rows = rows
        self.primes = primes
        self.wantA, self.wantB = oracle.cp_mm(P, A, B, primes, rows=rows)
        g = np.random.default_rng(seed)
        self.checks = []  # (prime index, part, r, P (X r))
        for i, q in enumerate(primes):
            Pq = oracle.residues_of_signed(P, q)
            for part, X in (("A", A[i]), ("B", B[i])):
                if X.shape[1] == 0:
                    continue
                for _ in range(vectors):
                    r = g.integers(0, q, size=X.shape[1], dtype=np.uint64)
                    self.checks.append((i, part, r, oracle.matvec_mod(q, Pq, oracle.matvec_mod(q, X, r))))

    def verify(self, PA, PB, what):
        for i, _ in enumerate(self.primes):
            assert np.array_equal(PA[i][self.rows], self.wantA[i][self.rows]), (what, i, "A rows")
            assert np.array_equal(PB[i][self.rows], self.wantB[i][self.rows]), (what, i, "B rows")
        for i, part, r, lhs in self.checks:
            C = PA[i] if part == "A" else PB[i]
            assert np.array_equal(oracle.matvec_mod(self.primes[i], C, r), lhs), (what, i, part, "Freivalds")


# ------------------------------------------------------------------------------------------
# d = 16384 over 2 primes
# ------------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def large16k():
    d, L = 16384, 2
    print(f"\n[configs] drawing d={d} L={L} on the device", flush=True)
    primes, P, A, B = wl.cpmm_uniform_device(1005, d, d, d, 50, L)
    hP, hA, hB = _host(P), _host(A), _host(B)
    print("[configs] oracle rows and Freivalds sides", flush=True)
    exp = _Expect(hP, hA, hB, primes, _rows(d), vectors=2, seed=16384)
    del hA, hB
    yield dict(d=d, primes=primes, P=P, A=A, B=B, exp=exp)
    del P, A, B
    torch.cuda.empty_cache()


@pytest.mark.parametrize("form", ["int8_crt", "int8"])
def test_cp_mm_d16384_two_primes(large16k, form):
    c = large16k
    print(f"\n[configs] cp_mm d={c['d']} L=2 form={form}", flush=True)
    PA, PB = hlb.cp_mm(c["P"], c["A"], c["B"], c["primes"], p_absmax=1 << 20, form=form)
    hPA, hPB = _host(PA), _host(PB)
    del PA, PB
    c["exp"].verify(hPA, hPB, form)


# ------------------------------------------------------------------------------------------
# The 64-problem batch over 4 primes of 45 bits
# ------------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def batch64():
    primes, shapes, probs = wl.batch_problems_device(1004, 64, 45, 4)
    print(f"\n[configs] batch of {len(probs)} problems, oracle sides", flush=True)
    expects = []
    for j, p in enumerate(probs):
        expects.append(_Expect(_host(p["P"]).view(np.int64), _host(p["A"]), _host(p["B"]), primes,
                               _rows(shapes[j][0]), vectors=1, seed=4000 + j))
    yield dict(primes=primes, shapes=shapes, probs=probs, expects=expects)
    del probs
    torch.cuda.empty_cache()


@pytest.mark.parametrize("form", ["int8_crt", "int8"])
def test_batch_64_uneven_problems(batch64, form):
    b = batch64
    L = len(b["primes"])
    print(f"\n[configs] cp_mm_batch 64 problems form={form}", flush=True)
    run = [dict(p, PA=torch.empty((L, m, d), dtype=torch.int64, device=DEV),
                PB=torch.empty((L, m, d), dtype=torch.int64, device=DEV))
           for p, (m, d) in zip(b["probs"], b["shapes"])]
    # twice: the first call captures the batch graph, the second replays it
    for rep in range(2):
        for r in run:
            r["PA"].fill_(-1)
            r["PB"].fill_(-1)
        hlb.cp_mm_batch(run, b["primes"], form=form)
        torch.cuda.synchronize()
        for j, (r, exp) in enumerate(zip(run, b["expects"])):
            exp.verify(_host(r["PA"]), _host(r["PB"]), (form, rep, j, b["shapes"][j]))


# ------------------------------------------------------------------------------------------
# End to end at d = 4096 over 3 primes, multimodular form
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("d,L,seed", [(4096, 3, 1002), (8192, 3, 1003), (16384, 2, 1005)])
def test_ckks_end_to_end_multimodular(d, L, seed):
    print(f"\n[configs] CKKS end to end d={d} L={L} int8_crt", flush=True)
    dr = wl.ckks_draws(seed=seed, m=d, k=d, n=d, bits=50, L=L)
    primes = dr.primes
    delta = 2.0 ** dr.delta_bits
    ME = oracle.encode(dr.M, delta) + dr.E                 # the encoded message plus error
    P = oracle.round_half_up(dr.U * 2.0 ** dr.p_scale_bits)
    gA = torch.from_numpy(dr.A.view(np.int64)).to(DEV)
    gS = torch.from_numpy(dr.S).to(DEV)
    gB = hlb.hlb_test_encrypt(gA, gS, torch.from_numpy(ME).to(DEV), primes)
    B = _host(gB)
    g = np.random.default_rng(d)
    # the ciphertext is a valid encryption: A S + B = encode(M) + E (mod q_i), by Freivalds
    for i, q in enumerate(primes):
        Sq = oracle.residues_of_signed(dr.S, q)
        MEq = oracle.residues_of_signed(ME, q)
        for _ in range(2):
            r = g.integers(0, q, size=d, dtype=np.uint64)
            lhs = (oracle.matvec_mod(q, dr.A[i], oracle.matvec_mod(q, Sq, r)) + oracle.matvec_mod(q, B[i], r)) % q
            assert np.array_equal(lhs, oracle.matvec_mod(q, MEq, r)), (i, "encryption")
    gP = torch.from_numpy(P).to(DEV)
    gPA, gPB = hlb.cp_mm(gP, gA, gB, primes, p_absmax=1 << dr.p_scale_bits, form="int8_crt")
    PA, PB = _host(gPA), _host(gPB)
    del gPA, gPB, gA, gB, gS, gP
    rows = _rows(d)
    _Expect(P, dr.A, B, primes, rows, vectors=2, seed=d + 1).verify(PA, PB, "ckks cp_mm")
    # decryption of the sampled rows: (P A) S + P B = P (encode(M) + E) (mod q_i), exactly
    D = oracle.decrypt(PA[:, rows], PB[:, rows], dr.S, primes)
    for i, q in enumerate(primes):
        want = oracle.mod_pp_mm(q, oracle.residues_of_signed(P[rows], q), oracle.residues_of_signed(ME, q))
        assert np.array_equal(D[i], want), (i, "decryption congruence")
    # the CRT lift is the exact integer product P (encode(M) + E) (|.| < 2^74 < Q / 2): formed
    # here from two exact int64 products over 20-bit halves of encode(M) + E
    lifted = oracle.crt_lift_centered(D, primes)
    lo = ME & ((1 << 20) - 1)
    hi = (ME - lo) >> 20
    exact = (P[rows] @ hi).astype(object) * (1 << 20) + (P[rows] @ lo).astype(object)
    assert lifted.tolist() == exact.tolist()
    # decoding: within k |P| (|E| + 1/2) / (Delta 2^20) of the cleartext product P M / 2^20
    scale = delta * 2.0 ** dr.p_scale_bits
    got = oracle.decode(lifted, scale)
    ref = (P[rows].astype(np.float64) @ dr.M) / 2.0 ** dr.p_scale_bits
    bound = d * np.abs(P).max() * (np.abs(dr.E).max() + 0.5) / scale
    assert np.abs(got - ref).max() <= bound
    assert oracle.precision_bits(ref, got) > 20
