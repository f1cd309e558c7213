"""GPU tests of CP-MM with a truncated b-part (Strategy 2 of Section 6.1), over one modulus.

INT8 form: the kernel skips the digit products of the low shifts; the result is a fixed
integer computation, so it must equal the oracle's truncated product bit for bit.  FP64
form: one floating-point product whose rounding depends on the summation order; it must lie
within the stated worst-case bound of the exact product (and of the oracle's own truncated
product), and be exact where no partial sum reaches 2^53.  In every case the a-part is exact.
"""
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


def _centred_diff(a, b, q):
    d = (a.astype(object) - b.astype(object)) % q
    return np.where(d > q // 2, d - q, d)


def _drop_budget(k, dx, drop):
    # the smallest budget that admits `drop` dropped shifts (it admits no more)
    pairs = lambda s: sum(1 for i in range(3) if 0 <= s - i < dx)
    return float(np.log2(k * 2 ** 14 * sum(pairs(s) * 256 ** s for s in range(drop)))) + 1e-6


@pytest.mark.parametrize("drop", [1, 2, 3])
@pytest.mark.parametrize("shape,bits", [((96, 300, 80), 50), ((60, 257, 130), 50), ((129, 190, 70), 45)])
def test_int8_drop_bit_exact_vs_oracle(drop, shape, bits):
    m, k, n = shape
    w = wl.cpmm_uniform(3000 + drop + m, m, k, n, bits, 1)
    budget = _drop_budget(k, 7 if bits == 50 else 6, drop)
    plan = hlb.plan_trunc_b(k, min(w.primes), max(w.primes), w.p_absmax, budget, "int8")
    assert plan["truncated"] and plan["dropped_shifts"] == drop
    PA, PB = hlb.cp_mm_trunc_b(_t(w.P), _t(w.A), _t(w.B), w.primes, budget, p_absmax=w.p_absmax,
                               form="int8")
    wantA, exactB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(_np(PA), wantA)
    gotB = _np(PB)
    dx = 7 if bits == 50 else 6
    for l, q in enumerate(w.primes):
        want = oracle.mod_pp_mm_drop_i8(q, w.P, w.B[l], drop, 3, dx)
        assert np.array_equal(gotB[l], want)
        assert np.abs(_centred_diff(gotB[l], exactB[l], q)).max() <= 2.0 ** plan["err_bound_log2"]


def test_budget_below_every_truncation_gives_the_exact_cp_mm():
    w = wl.cpmm_uniform(3100, 70, 200, 50, 50, 1)
    for form in ("int8", "fp64"):
        plan = hlb.plan_trunc_b(200, min(w.primes), max(w.primes), w.p_absmax, 10.0, form)
        assert not plan["truncated"]
        PA, PB = hlb.cp_mm_trunc_b(_t(w.P), _t(w.A), _t(w.B), w.primes, 10.0, p_absmax=w.p_absmax, form=form)
        wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
        assert np.array_equal(_np(PA), wantA) and np.array_equal(_np(PB), wantB)


@pytest.mark.parametrize("shape", [(64, 64, 64), (100, 513, 77), (33, 1000, 129), (100, 514, 78)])
def test_fp64_trunc_within_bound(shape):
    m, k, n = shape
    w = wl.cpmm_uniform(3200 + k, m, k, n, 50, 1)
    plan = hlb.plan_trunc_b(k, min(w.primes), max(w.primes), w.p_absmax, 60.0, "fp64")
    assert plan["truncated"] and plan["products"] == 1
    PA, PB = hlb.cp_mm_trunc_b(_t(w.P), _t(w.A), _t(w.B), w.primes, 60.0, p_absmax=w.p_absmax, form="fp64")
    wantA, exactB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(_np(PA), wantA)
    gotB = _np(PB)
    bound = 2.0 ** plan["err_bound_log2"]
    for l, q in enumerate(w.primes):
        err = np.abs(_centred_diff(gotB[l], exactB[l], q)).astype(float)
        assert err.max() <= bound
        # the oracle's truncated product obeys the same bound, so the two are within 2x of it
        ref = oracle.mod_pp_mm_trunc_fp64(q, w.P, w.B[l])
        assert np.abs(_centred_diff(gotB[l], ref, q)).astype(float).max() <= 2 * bound


def test_fp64_trunc_exact_regime():
    # k |P| q/2 < 2^53: the single FP64 product is exact, so the result is bit-exact
    g = wl.rng(3300)
    primes = [(1 << 31) - 1]
    m, k, n = 70, 96, 90
    P = g.integers(-(1 << 15), 1 << 15, size=(m, k))
    A = np.stack([g.integers(0, q, size=(k, n), dtype=np.uint64) for q in primes])
    B = np.stack([g.integers(0, q, size=(k, n), dtype=np.uint64) for q in primes])
    plan = hlb.plan_trunc_b(k, min(primes), max(primes), 1 << 15, 0.0, "fp64")
    assert plan["truncated"] and plan["err_bound_log2"] == float("-inf")
    PA, PB = hlb.cp_mm_trunc_b(_t(P), _t(A), _t(B), primes, 0.0, p_absmax=1 << 15, form="fp64")
    wantA, wantB = oracle.cp_mm(P, A, B, primes)
    assert np.array_equal(_np(PA), wantA) and np.array_equal(_np(PB), wantB)


def test_fp64_trunc_centring_on_device():
    # b-part all q - 1 (centred -1): exact even though uncentred products would round
    q = wl.ntt_primes(50, 1)[0]
    g = wl.rng(3301)
    m, k, n = 40, 4096, 20
    P = wl.plaintext_matrix(g, m, k)
    A = g.integers(0, q, size=(1, k, 8), dtype=np.uint64)
    B = np.full((1, k, n), q - 1, dtype=np.uint64)
    _, PB = hlb.cp_mm_trunc_b(_t(P), _t(A), _t(B), [q], 60.0, p_absmax=1 << 20, form="fp64")
    want = oracle.mod_pp_mm(q, oracle.residues_of_signed(P, q), B[0])
    assert np.array_equal(_np(PB)[0], want)


@pytest.mark.parametrize("form", ["int8", "fp64"])
def test_single_modulus_decryption_end_to_end(form):
    # The paper's setting: one modulus, a-part exact, b-part truncated.  With scales chosen so
    # that P (Delta M + E) stays below q / 2, decryption A' S + B' (mod q), lifted to the
    # centred representative, equals P (round(Delta M) + E) up to exactly the b-part error.
    d = wl.ckks_draws(seed=3400, m=48, k=1024, n=40, bits=50, L=1, delta_bits=20, p_scale_bits=15)
    q = d.primes[0]
    Menc = oracle.encode(d.M, 2.0 ** d.delta_bits)
    B = oracle.encrypt(d.A, d.S, Menc, d.E, d.primes)
    P = oracle.round_half_up(d.U * 2.0 ** d.p_scale_bits)
    exact = P.astype(object) @ (Menc + d.E).astype(object)
    assert np.abs(exact).max() < q // 2
    plan = hlb.plan_trunc_b(1024, q, q, 1 << 15, 40.0, form)
    assert plan["truncated"]
    PA, PB = hlb.cp_mm_trunc_b(_t(P), _t(d.A), _t(B), d.primes, 40.0, p_absmax=1 << 15, form=form)
    D = oracle.decrypt(_np(PA), _np(PB), d.S, d.primes)
    lifted = oracle.crt_lift_centered(D, d.primes)
    err = np.abs((lifted - exact).astype(float)).max()
    assert err <= 2.0 ** plan["err_bound_log2"]
    assert err > 0 or plan["err_bound_log2"] == float("-inf")


def test_more_than_one_modulus_is_rejected():
    w = wl.cpmm_uniform(3600, 16, 64, 16, 50, 2)
    with pytest.raises(hlb.HlbError):
        hlb.cp_mm_trunc_b(_t(w.P), _t(w.A), _t(w.B), w.primes, 45.0, p_absmax=w.p_absmax)


def test_large_int8_drop3_sampled_rows():
    # the launch configuration of the d = 4096 workload, checked on sampled output rows
    d = 4096
    w = wl.cpmm_uniform(3500, d, d, d, 50, 1)
    PA, PB = hlb.cp_mm_trunc_b(_t(w.P), _t(w.A), _t(w.B), w.primes, 45.0, p_absmax=w.p_absmax, form="int8")
    rows = [0, 1, 127, 128, 2047, 4000, 4095]
    gA, gB = _np(PA), _np(PB)
    assert hlb.plan_trunc_b(d, w.primes[0], w.primes[0], w.p_absmax, 45.0, "int8")["dropped_shifts"] == 3
    wantA, _ = oracle.cp_mm(w.P, w.A, w.B, w.primes, rows=rows)
    for l, q in enumerate(w.primes):
        assert np.array_equal(gA[l][rows], wantA[l][rows])
        want = oracle.mod_pp_mm_drop_i8(q, w.P[rows], w.B[l], 3, 3, 7)
        assert np.array_equal(gB[l][rows], want)
