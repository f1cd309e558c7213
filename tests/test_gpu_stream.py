"""GPU parity of the multimodular GEMM's persistent launch, where each workgroup runs many
tiles as one stream of pipeline stages and takes them from per-XCD queues (tile counts far
above the CU count, K-block counts of 4 -- the shortest tile the stream takes -- 6 and 32,
ragged m and n, and an odd count of 17 padded with a zero block to 18), and of the
one-tile-per-workgroup launch it falls back to (K-block counts odd and below 15, or below 4).

Every output matrix is checked against the oracle by Freivalds' test (P (X r) = C r mod q for
random r) and on sampled rows element by element; the products are also compared element by
element with the digit form, an independent exact path, which must give the same canonical
residues everywhere."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_16080_amd as hlb
import workloads as wl

pytestmark = pytest.mark.gpu


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("m,k,n,L", [
    (2048, 256, 2048, 3),   # 4 K blocks: 2816 tiles, the next tile learnt at the first group
    (1000, 384, 1500, 2),   # 6 K blocks, ragged rows and columns
    (777, 2000, 3000, 3),   # 32 K blocks (the last one partial)
    (1500, 1088, 1000, 2),  # 17 K blocks: odd, padded with a zero block to 18
    (1500, 576, 1000, 2),   # 9 K blocks: odd and short, one workgroup per tile
    (1500, 128, 1000, 2),   # 2 K blocks: shorter than the ring, one workgroup per tile
])
def test_stream_launch_vs_oracle_and_digit_form(m, k, n, L):
    print(f"\n[stream] m={m} k={k} n={n} L={L}", flush=True)
    primes, P, A, B = wl.cpmm_uniform_device(7000 + k, m, k, n, 50, L)
    PA, PB = hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form="int8_crt")
    DA, DB = hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form="int8")
    torch.cuda.synchronize()
    assert torch.equal(PA, DA) and torch.equal(PB, DB)
    hP = P.cpu().numpy()
    hA, hB = _host(A), _host(B)
    gA, gB = _host(PA), _host(PB)
    rows = sorted({0, 255, 256, m // 2 + 1, m - 1})
    wantA, wantB = oracle.cp_mm(hP, hA, hB, primes, rows=rows)
    g = np.random.default_rng(m + k + n)
    for i, q in enumerate(primes):
        assert np.array_equal(gA[i][rows], wantA[i][rows]), (i, "A rows")
        assert np.array_equal(gB[i][rows], wantB[i][rows]), (i, "B rows")
        Pq = oracle.residues_of_signed(hP, q)
        for X, C in ((hA[i], gA[i]), (hB[i], gB[i])):
            r = g.integers(0, q, size=n, dtype=np.uint64)
            lhs = oracle.matvec_mod(q, Pq, oracle.matvec_mod(q, X, r))
            assert np.array_equal(oracle.matvec_mod(q, C, r), lhs), (i, "Freivalds")


def test_stream_launch_back_to_back_shapes():
    """The queue counters start from zero on every call: a large call, then a smaller one on
    the same stream (same workspace), each checked against the digit form."""
    for (m, k, n, L) in [(1536, 512, 1536, 3), (640, 384, 700, 2)]:
        print(f"\n[stream] back to back m={m} k={k} n={n} L={L}", flush=True)
        primes, P, A, B = wl.cpmm_uniform_device(7100 + m, m, k, n, 45, L)
        PA, PB = hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form="int8_crt")
        DA, DB = hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form="int8")
        torch.cuda.synchronize()
        assert torch.equal(PA, DA) and torch.equal(PB, DB)
        rows = [0, m - 1]
        wantA, wantB = oracle.cp_mm(P.cpu().numpy(), _host(A), _host(B), primes, rows=rows)
        assert np.array_equal(_host(PA)[:, rows], wantA[:, rows])
        assert np.array_equal(_host(PB)[:, rows], wantB[:, rows])


@pytest.mark.parametrize("k,cls", [(16384, -1), (16448, -1), (16448, 1), (16512, -1), (131071, -1)])
def test_largest_products_closed_form(k, cls):
    """P = 128, A = 128 and B = q - 128 everywhere: modulo 256 every operand residue is -128, so
    each INT8 product reaches k 2^14 -- 2^28 at k = 16384, the deepest K whose products the
    epilogue reduces in single precision; 2^31 - 2^14 at k = 131071, the deepest the form takes.
    k = 16448 (257 K blocks, padded to 258) and 16512 run the general reduction in the
    persistent launch, and with the 256 x 256 tiles forced, one workgroup per tile.  Every
    output is 2^14 k (A part) or -2^14 k (B part) mod q."""
    print(f"\n[stream] largest products k={k} class={cls}", flush=True)
    primes = wl.ntt_primes(50, 1)
    q = primes[0]
    m, n = 256, 384
    P = torch.full((m, k), 128, dtype=torch.int64, device="cuda")
    A = torch.full((1, k, n), 128, dtype=torch.int64, device="cuda")
    B = torch.full((1, k, n), q - 128, dtype=torch.int64, device="cuda")
    try:
        hlb.set_option(hlb.OPT_CRT_WIDE, cls)
        PA, PB = hlb.cp_mm(P, A, B, primes, p_absmax=128, form="int8_crt")
    finally:
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
    gA, gB = _host(PA), _host(PB)
    assert (gA == (k << 14) % q).all()
    assert (gB == (-(k << 14)) % q).all()


@pytest.mark.parametrize("k,cls", [(16448, -1), (16448, 1), (20096, -1)])
def test_general_reduction_random_deep_k(k, cls):
    """Random operands past 256 K blocks, where the epilogue takes the general twelve-operation
    reduction: 257 blocks (padded to 258) and 314 in the persistent launch, and 257 with the
    256 x 256 tiles forced (one workgroup per tile).  Sampled rows against the oracle and every
    entry against the digit form."""
    print(f"\n[stream] general reduction k={k} class={cls}", flush=True)
    m, n, L = 300, 400, 2
    primes, P, A, B = wl.cpmm_uniform_device(7300 + k, m, k, n, 50, L)
    try:
        hlb.set_option(hlb.OPT_CRT_WIDE, cls)
        PA, PB = hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form="int8_crt")
    finally:
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
    DA, DB = hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form="int8")
    torch.cuda.synchronize()
    assert torch.equal(PA, DA) and torch.equal(PB, DB)
    rows = [0, 255, 256, m - 1]
    wantA, wantB = oracle.cp_mm(P.cpu().numpy(), _host(A), _host(B), primes, rows=rows)
    assert np.array_equal(_host(PA)[:, rows], wantA[:, rows])
    assert np.array_equal(_host(PB)[:, rows], wantB[:, rows])


def test_seeded_sweep_of_small_shapes():
    """Forty seeded shapes (m, k, n from 1 to 700, 1 to 4 primes, plaintext bounds from 1 to
    2^40): each against the oracle in full."""
    g = np.random.default_rng(7400)
    for i in range(40):
        m, k, n = (int(x) for x in g.integers(1, 700, size=3))
        L = int(g.integers(1, 5))
        pbits = int(g.integers(0, 41))
        print(f"\n[stream] sweep {i}: m={m} k={k} n={n} L={L} pbits={pbits}", flush=True)
        primes = wl.ntt_primes(int(g.integers(30, 53)), L, skip=i % 8)
        pmax = 1 << pbits
        P = g.integers(-pmax, pmax + 1, size=(m, k), dtype=np.int64)
        A = np.stack([g.integers(0, q, size=(k, n), dtype=np.uint64) for q in primes])
        B = np.stack([g.integers(0, q, size=(k, n), dtype=np.uint64) for q in primes])
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()
        PA, PB = hlb.cp_mm(t(P), t(A), t(B), primes, p_absmax=pmax, form="int8_crt")
        wantA, wantB = oracle.cp_mm(P, A, B, primes)
        assert np.array_equal(_host(PA), wantA), i
        assert np.array_equal(_host(PB), wantB), i
