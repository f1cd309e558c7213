"""GPU parity of the multimodular (CRT) INT8 form against the oracle, bit for bit.

The form computes the exact integer product modulo small coprime moduli and recombines it,
so its result is the unique canonical residue, like every other form: the oracle is the plain
definition of Mod-PP-MM / CP-MM."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_16080_amd as hlb
import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("wide", [2, 1, 0])
@pytest.mark.parametrize("dims", [(1, 1, 1, 1, 1), (33, 65, 17, 40, 1), (256, 128, 128, 128, 2),
                                  (200, 300, 130, 70, 3), (300, 64, 257, 1, 4), (64, 700, 64, 0, 2),
                                  (513, 129, 255, 129, 1), (100, 200, 600, 300, 1),
                                  # 18 output matrices: more than one GEMM launch's segments
                                  (70, 90, 40, 33, 9)])
def test_cp_mm_crt_vs_oracle(dims, wide):
    m, k, nA, nB, L = dims
    w = wl.cpmm_uniform(5000 + sum(dims), m, k, max(nA, nB, 1), 50, L)
    A, B = w.A[:, :, :nA], w.B[:, :, :nB]
    try:
        hlb.set_option(hlb.OPT_CRT_WIDE, wide)
        PA, PB = hlb.cp_mm(_t(w.P), _t(A), _t(B), w.primes, p_absmax=w.p_absmax, form="int8_crt")
        got = (_np(PA), _np(PB))
    finally:
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
    wantA, wantB = oracle.cp_mm(w.P, A, B, w.primes)
    assert np.array_equal(got[0], wantA) and np.array_equal(got[1], wantB)


def test_cp_mm_crt_45_bit_and_measured_bound():
    w = wl.cpmm_uniform(5100, 190, 333, 150, 45, 4)
    PA, PB = hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes, p_absmax=0, form="int8_crt")
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(_np(PA), wantA) and np.array_equal(_np(PB), wantB)


@pytest.mark.parametrize("q,D", [(2, 8), (3, 8), (97, 8), (65537, 8), ((1 << 31) - 1, 10), ((1 << 40) + 15, 12),
                                 ((1 << 45) + 59, 14), ((1 << 52) - 47, 16)])
def test_mod_pp_mm_crt_moduli(q, D):
    # both operands full residues: every instantiated moduli count
    g = wl.rng(q % 1000)
    m, k, n = 70, 200, 90
    assert hlb.plan(0, k, q, 1, "int8_crt")["p_limbs"] == D
    P = g.integers(0, q, size=(m, k), dtype=np.uint64)
    X = g.integers(0, q, size=(k, n), dtype=np.uint64)
    got = _np(hlb.mod_pp_mm(q, _t(P), _t(X), form="int8_crt"))
    assert np.array_equal(got, oracle.mod_pp_mm(q, P, X))


def test_crt_extreme_values_closed_form():
    # P = +-p_absmax and A = q - 1 everywhere: (P A)_ij = -sum_l P_il (mod q), exactly
    primes = wl.ntt_primes(50, 2)
    m, k, n = 40, 4096, 64
    for sign in (1, -1):
        P = np.full((m, k), sign * (1 << 20), dtype=np.int64)
        A = np.stack([np.full((k, n), q - 1, dtype=np.uint64) for q in primes])
        PA, PB = hlb.cp_mm(_t(P), _t(A), _t(A), primes, p_absmax=1 << 20, form="int8_crt")
        PA, PB = _np(PA), _np(PB)
        for i, q in enumerate(primes):
            want = (-sign * k * (1 << 20)) % q
            assert (PA[i] == want).all() and (PB[i] == want).all()
    # residues q - 1 on both sides (centred -1): every output is k mod q
    q = (1 << 52) - 47
    P = np.full((30, 3000), q - 1, dtype=np.uint64)
    got = _np(hlb.mod_pp_mm(q, _t(P), _t(P.T.copy()), form="int8_crt"))
    assert (got == 3000 % q).all()
    # residues (q-1)/2 and (q+1)/2: the two ends of the centred range
    X = np.full((3000, 20), (q + 1) // 2, dtype=np.uint64)
    P = np.full((30, 3000), (q - 1) // 2, dtype=np.uint64)
    got = _np(hlb.mod_pp_mm(q, _t(P), _t(X), form="int8_crt"))
    assert (got == oracle.mod_pp_mm(q, P[:1], X[:, :1])[0, 0]).all()


def test_ccmm_core_crt():
    primes = wl.ntt_primes(50, 2, skip=1)
    g = wl.rng(5200)
    m, k, n = 70, 130, 33
    A, B = (np.stack([wl.uniform_residues(g, (m, k), q) for q in primes]) for _ in range(2))
    At, Bt = (np.stack([wl.uniform_residues(g, (k, n), q) for q in primes]) for _ in range(2))
    got = hlb.ccmm_pp_core(_t(A), _t(B), _t(At), _t(Bt), primes, form="int8_crt")
    want = oracle.ccmm_pp_core(A, B, At, Bt, primes)
    for gC, wC in zip(got, want):
        assert np.array_equal(_np(gC), wC)


def test_crt_strided_and_edges():
    q = wl.ntt_primes(50, 1)[0]
    g = wl.rng(5300)
    Pb = g.integers(0, q, size=(50, 90), dtype=np.uint64)
    Xb = g.integers(0, q, size=(90, 70), dtype=np.uint64)
    P = _t(Pb)[:, 5:85]          # ldp = 90, k = 80
    X = _t(Xb)[5:85, 3:60]       # ldx = 70, n = 57
    got = _np(hlb.mod_pp_mm(q, P, X, form="int8_crt"))
    assert np.array_equal(got, oracle.mod_pp_mm(q, Pb[:, 5:85], Xb[5:85, 3:60]))
    # k = 0 writes zeros
    C = hlb.mod_pp_mm(q, torch.zeros((5, 0), dtype=torch.int64, device=DEV),
                      torch.zeros((0, 7), dtype=torch.int64, device=DEV), form="int8_crt")
    assert (_np(C) == 0).all()


def test_crt_large_sampled_rows_and_forms_agree():
    # the d = 4096 shape: sampled rows against the oracle, and the three forms bit-identical
    d = 4096
    w = wl.cpmm_uniform(5400, d, d, d, 50, 2)
    rows = [0, 1, 255, 256, 2047, 4000, 4095]
    out = {}
    for form in ("int8_crt", "int8"):
        PA, PB = hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes, p_absmax=w.p_absmax, form=form)
        out[form] = (_np(PA), _np(PB))
    assert np.array_equal(out["int8_crt"][0], out["int8"][0])
    assert np.array_equal(out["int8_crt"][1], out["int8"][1])
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes, rows=rows)
    for l in range(2):
        assert np.array_equal(out["int8_crt"][0][l][rows], wantA[l][rows])
        assert np.array_equal(out["int8_crt"][1][l][rows], wantB[l][rows])


def test_auto_picks_form_by_shape():
    # AUTO: the multimodular GEMM for products of at least 256 x 256 outputs, the digit GEMM
    # below that (the kernels that ran are visible in the profiling records)
    w = wl.cpmm_uniform(5500, 512, 300, 512, 50, 1)
    small = wl.cpmm_uniform(5501, 100, 300, 80, 50, 1)
    ran = {}
    try:
        for name, case in (("big", w), ("small", small)):
            hlb.profile_reset()
            hlb.set_option(hlb.OPT_PROFILE, 1)
            PA, PB = hlb.cp_mm(_t(case.P), _t(case.A), _t(case.B), case.primes, p_absmax=case.p_absmax, form="auto")
            torch.cuda.synchronize()
            hlb.set_option(hlb.OPT_PROFILE, 0)
            ran[name] = {k: hlb.profile_read(k)[0] for k in ("crt_gemm", "gemm_i8")}
            want = oracle.cp_mm(case.P, case.A, case.B, case.primes)
            assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1])
    finally:
        hlb.set_option(hlb.OPT_PROFILE, 0)
        hlb.profile_reset()
    assert ran["big"] == {"crt_gemm": 1, "gemm_i8": 0}
    assert ran["small"] == {"crt_gemm": 0, "gemm_i8": 1}


def test_batch_in_multimodular_form():
    # a batch in the multimodular form: one batched split, GEMM and recombination launch
    primes = wl.ntt_primes(45, 2)
    g = wl.rng(5600)
    probs, want = [], []
    for m, k, n in ((300, 200, 260), (64, 128, 96), (257, 513, 300)):
        P = wl.plaintext_matrix(g, m, k)
        A = np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])
        B = np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])
        probs.append(dict(P=_t(P), A=_t(A), B=_t(B), p_absmax=1 << 20,
                          PA=torch.empty((2, m, n), dtype=torch.int64, device=DEV),
                          PB=torch.empty((2, m, n), dtype=torch.int64, device=DEV)))
        want.append(oracle.cp_mm(P, A, B, primes))
    hlb.cp_mm_batch(probs, primes, form="int8_crt")
    for p, (wA, wB) in zip(probs, want):
        assert np.array_equal(_np(p["PA"]), wA) and np.array_equal(_np(p["PB"]), wB)


@pytest.mark.parametrize("graph", [1, 0])
def test_batch_multimodular_replays_and_degenerate_members(graph):
    # graph-cached and eager batches; a replay after the inputs change (same pointers) must
    # follow them; members with k = 0, m = 0, one empty part, and sizes off every tile edge
    primes = wl.ntt_primes(50, 3, skip=2)
    g = wl.rng(5800 + graph)
    shapes = [(130, 70, 33, 257), (0, 64, 64, 64), (65, 0, 40, 40), (300, 129, 0, 130), (257, 1000, 500, 0),
              (33, 64, 300, 1)]
    host, probs = [], []
    for m, k, nA, nB in shapes:
        P = wl.plaintext_matrix(g, m, k)
        A = np.stack([wl.uniform_residues(g, (k, nA), q) for q in primes])
        B = np.stack([wl.uniform_residues(g, (k, nB), q) for q in primes])
        host.append([P, A, B])
        probs.append(dict(P=_t(P), A=_t(A), B=_t(B), p_absmax=1 << 20,
                          PA=torch.full((3, m, nA), -1, dtype=torch.int64, device=DEV),
                          PB=torch.full((3, m, nB), -1, dtype=torch.int64, device=DEV)))
    hlb.set_option(hlb.OPT_BATCH_GRAPH, graph)
    try:
        for rnd in range(2):
            if rnd == 1:
                # new values in the same buffers
                for (P, A, B), pr in zip(host, probs):
                    P[...] = wl.plaintext_matrix(g, *P.shape)
                    for i, q in enumerate(primes):
                        A[i] = wl.uniform_residues(g, A.shape[1:], q)
                        B[i] = wl.uniform_residues(g, B.shape[1:], q)
                    pr["P"].copy_(_t(P))
                    pr["A"].copy_(_t(A))
                    pr["B"].copy_(_t(B))
            hlb.cp_mm_batch(probs, primes, form="int8_crt")
            for (P, A, B), pr in zip(host, probs):
                wA, wB = oracle.cp_mm(P, A, B, primes)
                assert np.array_equal(_np(pr["PA"]), wA) and np.array_equal(_np(pr["PB"]), wB)
    finally:
        hlb.set_option(hlb.OPT_BATCH_GRAPH, 1)


def test_batch_multimodular_moduli_count_from_largest_member():
    # one member with a 40-bit plaintext sets the batch's moduli count (14 instead of 10);
    # every member, also the 20-bit ones, must stay exact with it
    primes = wl.ntt_primes(50, 2, skip=4)
    g = wl.rng(5900)
    shapes = [(100, 300, 70, 130, 20), (257, 64, 300, 33, 40), (64, 129, 64, 64, 20)]
    assert hlb.plan(1, 300, max(primes), 1 << 40, "int8_crt")["p_limbs"] == 14
    probs, want = [], []
    for m, k, nA, nB, bits in shapes:
        P = wl.plaintext_matrix(g, m, k, scale_bits=bits)
        A = np.stack([wl.uniform_residues(g, (k, nA), q) for q in primes])
        B = np.stack([wl.uniform_residues(g, (k, nB), q) for q in primes])
        probs.append(dict(P=_t(P), A=_t(A), B=_t(B), p_absmax=1 << bits,
                          PA=torch.empty((2, m, nA), dtype=torch.int64, device=DEV),
                          PB=torch.empty((2, m, nB), dtype=torch.int64, device=DEV)))
        want.append(oracle.cp_mm(P, A, B, primes))
    hlb.cp_mm_batch(probs, primes, form="int8_crt")
    for p, (wA, wB) in zip(probs, want):
        assert np.array_equal(_np(p["PA"]), wA) and np.array_equal(_np(p["PB"]), wB)


@pytest.mark.parametrize("graph", [1, 0])
def test_batch_multimodular_tile_classes_from_the_table(graph):
    # tuning-table entries give the members three different tile classes, so the batch runs
    # one persistent GEMM launch per class; a forced class then overrides the table; every
    # member exact each time
    primes = wl.ntt_primes(45, 2, skip=1)
    g = wl.rng(6000 + graph)
    shapes = [(300, 200, 260), (600, 130, 400), (70, 520, 90), (1100, 64, 700)]
    probs, want = [], []
    for m, k, n in shapes:
        P = wl.plaintext_matrix(g, m, k)
        A = np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])
        B = np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])
        probs.append(dict(P=_t(P), A=_t(A), B=_t(B), p_absmax=1 << 20,
                          PA=torch.empty((2, m, n), dtype=torch.int64, device=DEV),
                          PB=torch.empty((2, m, n), dtype=torch.int64, device=DEV)))
        want.append(oracle.cp_mm(P, A, B, primes))
    D = hlb.plan(1, max(k for _, k, _ in shapes), max(primes), 1 << 20, "int8_crt")["p_limbs"]
    keys = [(D, int(np.log2(m)), int(np.log2(n)), int(np.log2(k))) for m, k, n in shapes]
    assert len(set(keys)) == len(keys)
    hlb.set_option(hlb.OPT_BATCH_GRAPH, graph)
    try:
        for key, cls in zip(keys, (0, 1, 2, 0)):
            hlb.hlb_tune_set_crt(*key, cls)
        assert [hlb.hlb_tune_class_crt(D, m, n, k) for m, k, n in shapes] == [0, 1, 2, 0]
        for forced in (-1, 1):
            hlb.set_option(hlb.OPT_CRT_WIDE, forced)
            for p in probs:
                p["PA"].fill_(-1)
                p["PB"].fill_(-1)
            hlb.cp_mm_batch(probs, primes, form="int8_crt")
            for j, (p, (wA, wB)) in enumerate(zip(probs, want)):
                assert np.array_equal(_np(p["PA"]), wA) and np.array_equal(_np(p["PB"]), wB), (forced, j)
    finally:
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
        hlb.set_option(hlb.OPT_BATCH_GRAPH, 1)
        for key in keys:
            hlb.hlb_tune_set_crt(*key, -1)
