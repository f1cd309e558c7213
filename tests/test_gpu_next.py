"""GPU tests of the rows beyond the core CP-MM: the CC-MM plaintext core (four Mod-PP-MMs
with shared digit splits), the exact RNS Rescale that ends Algorithm alg:pcmm, and the
online step of CP-MM with precomputation (the b-part product alone)."""
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


@pytest.mark.parametrize("form", ["int8", "fp64"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (70, 130, 33), (129, 257, 100)])
def test_ccmm_pp_core_vs_oracle(form, shape):
    m, k, n = shape
    primes = wl.ntt_primes(50, 2, skip=1)
    g = wl.rng(sum(shape))
    A, B = (np.stack([wl.uniform_residues(g, (m, k), q) for q in primes]) for _ in range(2))
    At, Bt = (np.stack([wl.uniform_residues(g, (k, n), q) for q in primes]) for _ in range(2))
    got = hlb.ccmm_pp_core(_t(A), _t(B), _t(At), _t(Bt), primes, form=form)
    want = oracle.ccmm_pp_core(A, B, At, Bt, primes)
    for gC, wC in zip(got, want):
        assert np.array_equal(_np(gC), wC)


def test_rescale_vs_oracle_and_edges():
    primes = wl.ntt_primes(50, 4)
    g = wl.rng(77)
    X = np.stack([wl.uniform_residues(g, (300, 70), q) for q in primes])
    q = primes[-1]
    # plant the rounding edges in the last residue: 0, (q-1)/2, (q+1)/2, q-1
    X[-1, 0, :4] = [0, (q - 1) // 2, (q + 1) // 2, q - 1]
    got = _np(hlb.rescale(_t(X), primes))
    assert np.array_equal(got, oracle.rescale(X, primes))


@pytest.mark.parametrize("form", ["int8_crt", "int8"])
def test_cp_mm_then_rescale_decrypts_to_scaled_product(form):
    # Algorithm alg:pcmm end to end: ct over L primes -> (P A, P B) -> Rescale by the last
    # prime q_L -> decryption under the same secret with the first L-1 primes gives
    # P (encode(M) + E) / q_L up to the rescaling error, i.e. k |S| / 2 + 1/2 per entry.
    d = wl.ckks_draws(seed=2101, m=40, k=128, n=48, bits=50, L=4)
    delta = 2.0 ** d.delta_bits
    Menc = oracle.encode(d.M, delta)
    B = oracle.encrypt(d.A, d.S, Menc, d.E, d.primes)
    P = oracle.round_half_up(d.U * 2.0 ** d.p_scale_bits)
    PA, PB = hlb.cp_mm(_t(P), _t(d.A), _t(B), d.primes, p_absmax=1 << d.p_scale_bits, form=form)
    rA, rB = hlb.rescale(PA, d.primes), hlb.rescale(PB, d.primes)
    # the rescaled parts equal the oracle's rescale of the oracle's product, bit for bit
    oA, oB = oracle.cp_mm(P, d.A, B, d.primes)
    assert np.array_equal(_np(rA), oracle.rescale(oA, d.primes))
    assert np.array_equal(_np(rB), oracle.rescale(oB, d.primes))
    primes2 = d.primes[:-1]
    D = oracle.decrypt(_np(rA), _np(rB), d.S, primes2)
    lifted = oracle.crt_lift_centered(D, primes2)
    exact = (P.astype(object) @ (Menc + d.E).astype(object))
    q = d.primes[-1]
    n = d.S.shape[0]
    err = np.abs((lifted * q - exact).astype(float)).max() / q
    assert err <= n * 1 * 0.5 + 0.5 + 1e-9   # rounding of A' and B' by at most 1/2 each


@pytest.mark.parametrize("form", ["int8_crt", "int8", "fp64"])
def test_precomputation_online_step_is_b_part_only(form):
    # CP-MM with precomputation: the online work is the single product B' = P B per prime
    # (nA = 0), bit-identical to the b-part of the full CP-MM.
    w = wl.cpmm_uniform(2201, 96, 300, 80, 50, 3)
    empty = torch.zeros((3, 300, 0), dtype=torch.int64, device=DEV)
    _, PB = hlb.cp_mm(_t(w.P), empty, _t(w.B), w.primes, p_absmax=w.p_absmax, form=form)
    _, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(_np(PB), wantB)
