"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Every result of the library is a canonical residue in [0, q), and exactly one correct value
exists, so all comparisons are exact equality.  Inputs come from the seeded generators in
``workloads``; expected values only from ``oracle``.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_16080_amd as hlb
import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda"
FORMS = ["int8", "fp64"]


def _t(a):
    """numpy integer array -> int64 CUDA tensor (uint64 bits preserved)."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def _mod_pp_mm_case(seed, m, k, n, bits, form):
    g = wl.rng(seed)
    q = wl.ntt_primes(bits, 1, skip=seed % 8)[0]
    P = wl.uniform_residues(g, (m, k), q)
    X = wl.uniform_residues(g, (k, n), q)
    got = _np(hlb.mod_pp_mm(q, _t(P), _t(X), form=form))
    want = oracle.mod_pp_mm(q, P, X)
    return got, want


@pytest.mark.parametrize("form", FORMS)
def test_mod_pp_mm_plain_256(form):
    # the 256 x 256 x 256 single-prime Mod-PP-MM (full residues on both sides)
    got, want = _mod_pp_mm_case(1001, 256, 256, 256, 50, form)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 33, 5), (65, 130, 63), (130, 257, 129),
                                   (64, 64, 64), (257, 100, 3), (3, 520, 200)])
def test_mod_pp_mm_ragged(form, shape):
    m, k, n = shape
    got, want = _mod_pp_mm_case(7 + m + k + n, m, k, n, 52, form)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("q", [2, 3, 97, 65537, (1 << 31) - 1, (1 << 52) - 47])
def test_mod_pp_mm_moduli(form, q):
    g = wl.rng(q % 1000)
    P = wl.uniform_residues(g, (40, 90), q)
    X = wl.uniform_residues(g, (90, 70), q)
    got = _np(hlb.mod_pp_mm(q, _t(P), _t(X), form=form))
    assert np.array_equal(got, oracle.mod_pp_mm(q, P, X))


@pytest.mark.parametrize("form", FORMS)
def test_mod_pp_mm_all_q_minus_one(form):
    # (q-1)^2 = 1 mod q, so every output equals k mod q: catches carry/sign slips in
    # the split, the limb products and the recombination at extreme digits
    q = wl.ntt_primes(52, 1)[0]
    for k in [1, 63, 64, 65, 1000]:
        P = np.full((70, k), q - 1, dtype=np.uint64)
        X = np.full((k, 66), q - 1, dtype=np.uint64)
        got = _np(hlb.mod_pp_mm(q, _t(P), _t(X), form=form))
        assert (got == k % q).all(), k


def test_mod_pp_mm_strided_operands():
    q = wl.ntt_primes(50, 1)[0]
    g = wl.rng(5)
    Pbig = wl.uniform_residues(g, (50, 80), q)
    Xbig = wl.uniform_residues(g, (70, 90), q)
    P, X = Pbig[:, :70], Xbig[:, :60]
    for form in FORMS:
        C = torch.zeros((50, 75), dtype=torch.int64, device=DEV)
        hlb.mod_pp_mm(q, _t(Pbig)[:, :70], _t(Xbig)[:, :60], form=form, out=C[:, :60])
        got = _np(C)
        assert np.array_equal(got[:, :60], oracle.mod_pp_mm(q, P, X))
        assert (got[:, 60:] == 0).all()


def _cpmm_case(seed, m, k, nA, nB, bits, L, form, p_absmax=None):
    w = wl.cpmm_uniform(seed, m, k, nA, bits, L, nB=nB)
    pm = w.p_absmax if p_absmax is None else p_absmax
    PA, PB = hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes, p_absmax=pm, form=form)
    return w, _np(PA), _np(PB)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dims", [(1, 1, 1, 1, 1), (33, 65, 17, 40, 1), (128, 128, 64, 64, 2),
                                  (200, 300, 130, 70, 3), (129, 64, 257, 1, 4), (64, 700, 64, 0, 2)])
def test_cp_mm_vs_oracle(form, dims):
    m, k, nA, nB, L = dims
    w, PA, PB = _cpmm_case(100 + sum(dims), m, k, nA, nB, 50, L, form)
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(PA, wantA)
    assert np.array_equal(PB, wantB)


def test_cp_mm_forms_bit_identical_and_45_bit_primes():
    w, PA8, PB8 = _cpmm_case(77, 190, 333, 150, 150, 45, 4, "int8")
    _, PA64, PB64 = _cpmm_case(77, 190, 333, 150, 150, 45, 4, "fp64")
    assert np.array_equal(PA8, PA64) and np.array_equal(PB8, PB64)
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(PA8, wantA) and np.array_equal(PB8, wantB)


@pytest.mark.parametrize("form", FORMS)
def test_cp_mm_measured_bound_and_large_plaintext(form):
    # p_absmax = 0: the library measures max |P| on the device
    w, PA, PB = _cpmm_case(91, 96, 200, 80, 80, 50, 2, form, p_absmax=0)
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(PA, wantA) and np.array_equal(PB, wantB)
    # a plaintext beyond three int8 digits (|P| up to 2^40) takes the wider plan
    g = wl.rng(92)
    P = g.integers(-(1 << 40), (1 << 40) + 1, size=(70, 150), dtype=np.int64)
    PA, PB = hlb.cp_mm(_t(P), _t(w.A[:, :150]), _t(w.B[:, :150]), w.primes, p_absmax=1 << 40, form=form)
    wantA, wantB = oracle.cp_mm(P, w.A[:, :150], w.B[:, :150], w.primes)
    assert np.array_equal(_np(PA), wantA) and np.array_equal(_np(PB), wantB)


@pytest.mark.parametrize("form", FORMS)
def test_cp_mm_extreme_plaintext_closed_form(form):
    # P = +-p_absmax everywhere and A = q - 1: (P A)_ij = -sum_l P_il (mod q), computed here
    # with Python integers; k spans many K stages, so every accumulator sees extreme digits.
    primes = wl.ntt_primes(50, 2)
    m, k, n = 40, 4096, 64
    for sign in (1, -1):
        P = np.full((m, k), sign * (1 << 20), dtype=np.int64)
        A = np.stack([np.full((k, n), q - 1, dtype=np.uint64) for q in primes])
        PA, PB = hlb.cp_mm(_t(P), _t(A), _t(A), primes, p_absmax=1 << 20, form=form)
        PA, PB = _np(PA), _np(PB)
        for i, q in enumerate(primes):
            want = (-sign * k * (1 << 20)) % q
            assert (PA[i] == want).all() and (PB[i] == want).all()


@pytest.mark.parametrize("form", FORMS)
def test_cp_mm_forced_k_chunk_fold(form):
    # force K folding every 128 elements (exactness plan of a much longer K) and compare
    w = wl.cpmm_uniform(61, 100, 1000, 90, 50, 3)
    try:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 128)
        PA, PB = hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes, p_absmax=w.p_absmax, form=form)
        got = (_np(PA), _np(PB))
    finally:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 0)
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(got[0], wantA) and np.array_equal(got[1], wantB)


def test_mod_pp_mm_forced_fold_general_form():
    q = wl.ntt_primes(52, 1)[0]
    g = wl.rng(62)
    P = wl.uniform_residues(g, (66, 700), q)
    X = wl.uniform_residues(g, (700, 65), q)
    try:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 64)
        got = {f: _np(hlb.mod_pp_mm(q, _t(P), _t(X), form=f)) for f in FORMS}
    finally:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 0)
    want = oracle.mod_pp_mm(q, P, X)
    for f in FORMS:
        assert np.array_equal(got[f], want), f


def test_edge_shapes():
    q = wl.ntt_primes(50, 1)[0]
    primes = [q]
    # k = 0 writes zeros
    C = torch.full((5, 6), 7, dtype=torch.int64, device=DEV)
    P = torch.zeros((5, 0), dtype=torch.int64, device=DEV)
    X = torch.zeros((0, 6), dtype=torch.int64, device=DEV)
    for form in FORMS:
        hlb.mod_pp_mm(q, P, X, form=form, out=C)
        assert (_np(C) == 0).all()
    # ... only inside a strided output: the columns around it keep their values
    for form in FORMS:
        big = torch.full((5, 9), 7, dtype=torch.int64, device=DEV)
        hlb.mod_pp_mm(q, P, X, form=form, out=big[:, 1:7])
        b = _np(big)
        assert (b[:, 1:7] == 0).all() and (b[:, 0] == 7).all() and (b[:, 7:] == 7).all()
    A = torch.zeros((1, 0, 6), dtype=torch.int64, device=DEV)
    PA, PB = hlb.cp_mm(P, A, A, primes, p_absmax=1, form="int8")
    assert (_np(PA) == 0).all() and (_np(PB) == 0).all()
    # m = 0, n = 0 and L = 0 are no-ops
    hlb.mod_pp_mm(q, torch.zeros((0, 4), dtype=torch.int64, device=DEV),
                  torch.zeros((4, 3), dtype=torch.int64, device=DEV))
    hlb.cp_mm(torch.zeros((3, 4), dtype=torch.int64, device=DEV),
              torch.zeros((0, 4, 2), dtype=torch.int64, device=DEV),
              torch.zeros((0, 4, 2), dtype=torch.int64, device=DEV), [], p_absmax=1)


def test_validate_and_absmax():
    q = wl.ntt_primes(50, 1)[0]
    g = wl.rng(9)
    X = wl.uniform_residues(g, (300, 200), q)
    assert hlb.validate_residues(_t(X), q) == -1
    X[123, 45] = q
    X[200, 7] = q + 5
    assert hlb.validate_residues(_t(X), q) == 123 * 200 + 45
    P = wl.plaintext_matrix(g, 100, 333)
    P[17, 5] = -(1 << 30)
    assert hlb.plaintext_absmax(_t(P)) == 1 << 30


def test_determinism():
    w = wl.cpmm_uniform(71, 256, 512, 192, 50, 3)
    outs = [hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes, p_absmax=w.p_absmax, form="int8")
            for _ in range(3)]
    ref = (_np(outs[0][0]), _np(outs[0][1]))
    for PA, PB in outs[1:]:
        assert np.array_equal(_np(PA), ref[0]) and np.array_equal(_np(PB), ref[1])


def test_determinism_across_runs_tile_classes_and_forms():
    """Bytes identical over repeated calls (the persistent multimodular launch takes its tiles
    from atomic queues, in an order that changes from run to run), over every tile class of
    both INT8 forms, and across the three forms.  1024 x 512 x 1536 over 3 primes: 528
    multimodular tiles of 256 x 384, more than one per CU."""
    w = wl.cpmm_uniform(72, 1024, 512, 1536, 50, 3)
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    outs = []
    try:
        for cls in (2, 2, 2, 1, 0):
            hlb.set_option(hlb.OPT_CRT_WIDE, cls)
            outs.append(hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form="int8_crt"))
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
        for cls in (0, 1):
            hlb.set_option(hlb.OPT_FORCE_CLASS, cls)
            outs.append(hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form="int8"))
        hlb.set_option(hlb.OPT_FORCE_CLASS, -1)
        outs.append(hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form="fp64"))
    finally:
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
        hlb.set_option(hlb.OPT_FORCE_CLASS, -1)
    ref = (_np(outs[0][0]), _np(outs[0][1]))
    for i, (PA, PB) in enumerate(outs[1:]):
        assert np.array_equal(_np(PA), ref[0]) and np.array_equal(_np(PB), ref[1]), i
    rows = [0, 255, 256, 1023]
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes, rows=rows)
    assert np.array_equal(ref[0][:, rows], wantA[:, rows]) and np.array_equal(ref[1][:, rows], wantB[:, rows])


@pytest.mark.parametrize("form", ["int8_crt", "int8", "fp64"])
def test_plaintext_on_the_right_by_transposition(form):
    """The paper's CP-MM returns an encryption of M U, the ciphertext parts times a plaintext on
    the right (Section 2's problem statement; Eq LZoutput: (A U, B U)).  The library multiplies
    the plaintext on the left, and (A U)^t = U^t A^t gives the right product from the transposed
    operands; checked in full against the oracle's A U mod q, with a plaintext shared by both
    parts and every prime."""
    d1, d2, d3, L = 300, 500, 200, 2
    primes = wl.ntt_primes(50, L, skip=3)
    g = wl.rng(7500)
    A = np.stack([wl.uniform_residues(g, (d1, d2), q) for q in primes])
    B = np.stack([wl.uniform_residues(g, (d1, d2), q) for q in primes])
    U = wl.plaintext_matrix(g, d2, d3)
    tr = lambda X: np.ascontiguousarray(np.transpose(X, (0, 2, 1)))
    PA, PB = hlb.cp_mm(_t(np.ascontiguousarray(U.T)), _t(tr(A)), _t(tr(B)), primes,
                       p_absmax=int(np.abs(U).max()), form=form)
    gotA, gotB = tr(_np(PA)), tr(_np(PB))
    for i, q in enumerate(primes):
        Uq = oracle.residues_of_signed(U, q)
        assert np.array_equal(gotA[i], oracle.mod_pp_mm(q, A[i], Uq)), (i, "A U")
        assert np.array_equal(gotB[i], oracle.mod_pp_mm(q, B[i], Uq)), (i, "B U")
