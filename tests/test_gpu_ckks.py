"""End-to-end CKKS checks of the GPU CP-MM: a real encryption (built by the oracle's
helpers), the GPU product, and decryption -- plus the library's test-only helpers against the
oracle's."""
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


@pytest.mark.parametrize("form", ["int8_crt", "int8", "fp64"])
def test_encrypted_product_decrypts_to_plaintext_product(form):
    # ct = (A, B) with A S + B = encode(M) + E (mod q_i); after CP-MM,
    # (P A) S + P B = P (encode(M) + E) (mod q_i) exactly, and decoding gives P M within the
    # noise bound k |P| (|E| + 1/2) / (Delta 2^20).
    d = wl.ckks_draws(seed=2002, m=48, k=256, n=40, bits=50, L=3)
    delta = 2.0 ** d.delta_bits
    Menc = oracle.encode(d.M, delta)
    B = oracle.encrypt(d.A, d.S, Menc, d.E, d.primes)
    P = oracle.round_half_up(d.U * 2.0 ** d.p_scale_bits)
    PA, PB = hlb.cp_mm(_t(P), _t(d.A), _t(B), d.primes, p_absmax=1 << d.p_scale_bits, form=form)
    D = oracle.decrypt(_np(PA), _np(PB), d.S, d.primes)
    lifted = oracle.crt_lift_centered(D, d.primes)
    exact = P.astype(object) @ (Menc + d.E).astype(object)
    assert lifted.tolist() == exact.tolist()
    got = oracle.decode(lifted, delta * 2.0 ** d.p_scale_bits)
    ref = (P.astype(np.float64) @ d.M) / 2.0 ** d.p_scale_bits
    k = d.M.shape[0]
    bound = k * np.abs(P).max() * (np.abs(d.E).max() + 0.5) / (delta * 2.0 ** d.p_scale_bits)
    assert np.abs(got - ref).max() <= bound
    assert oracle.precision_bits(ref, got) > 20


def test_library_test_helpers_match_oracle():
    d = wl.ckks_draws(seed=2003, m=8, k=96, n=72, bits=50, L=3)
    delta = 2.0 ** d.delta_bits
    Menc = oracle.encode(d.M, delta)
    got_enc = hlb.hlb_test_encode(torch.from_numpy(d.M).to(DEV), delta)
    assert np.array_equal(got_enc.cpu().numpy(), Menc)
    B_want = oracle.encrypt(d.A, d.S, Menc, d.E, d.primes)
    B = hlb.hlb_test_encrypt(_t(d.A), _t(d.S), _t(Menc + d.E), d.primes)
    assert np.array_equal(_np(B), B_want)
    D = hlb.hlb_test_decrypt(_t(d.A), B, _t(d.S), d.primes)
    assert np.array_equal(_np(D), oracle.decrypt(d.A, B_want, d.S, d.primes))
    for i, q in enumerate(d.primes):
        assert np.array_equal(_np(D)[i], ((Menc + d.E) % q).astype(np.uint64))
