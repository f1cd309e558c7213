"""GPU parity of the two FP64-form paths: prepared double planes + direct-to-LDS GEMM (plans
with one plaintext limb) and the register-staged kernel.  Each case runs with the plane path
on and off; both must equal the oracle bit for bit."""
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


def _both_paths(fn):
    out = []
    try:
        for direct in (1, 0):
            hlb.set_option(hlb.OPT_F64_PLANES, direct)
            out.append(fn())
    finally:
        hlb.set_option(hlb.OPT_F64_PLANES, 1)
    return out


# even shapes take the direct kernel: ragged in every dimension, a single stage, many stages,
# the smallest even K and N
@pytest.mark.parametrize("dims", [(1, 2, 2, 2, 1), (65, 18, 130, 66, 2), (100, 130, 66, 64, 3),
                                  (64, 16, 64, 64, 1), (200, 1000, 194, 130, 2), (3, 4096, 8, 2, 1)])
def test_cp_mm_fp64_direct_and_staged_vs_oracle(dims):
    m, k, nA, nB, L = dims
    w = wl.cpmm_uniform(4000 + sum(dims), m, k, max(nA, nB), 50, L)
    A, B = w.A[:, :, :nA], w.B[:, :, :nB]
    run = lambda: tuple(_np(x) for x in hlb.cp_mm(_t(w.P), _t(A), _t(B), w.primes, p_absmax=w.p_absmax,
                                                      form="fp64"))
    want = oracle.cp_mm(w.P, A, B, w.primes)
    for got in _both_paths(run):
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_cp_mm_fp64_direct_with_fold_and_four_limbs():
    # forced K folds through the direct kernel; a wider plaintext bound gives 4 limbs
    w = wl.cpmm_uniform(4100, 96, 1200, 80, 50, 2)
    want = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    try:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 128)
        got = _both_paths(lambda: tuple(_np(x) for x in hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes,
                                                                   p_absmax=w.p_absmax, form="fp64")))
    finally:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 0)
    for g in got:
        assert np.array_equal(g[0], want[0]) and np.array_equal(g[1], want[1])
    g = wl.rng(4101)
    P = g.integers(-(1 << 36), (1 << 36) + 1, size=(70, 300), dtype=np.int64)
    plan = hlb.plan(1, 300, max(w.primes), 1 << 36, "fp64")
    assert plan["p_limbs"] == 1 and plan["x_limbs"] == 4
    want = oracle.cp_mm(P, w.A[:, :300], w.B[:, :300], w.primes)
    got = _both_paths(lambda: tuple(_np(x) for x in hlb.cp_mm(_t(P), _t(w.A[:, :300]), _t(w.B[:, :300]),
                                                               w.primes, p_absmax=1 << 36, form="fp64")))
    for gg in got:
        assert np.array_equal(gg[0], want[0]) and np.array_equal(gg[1], want[1])


def test_fp64_misaligned_and_odd_strides():
    # plaintext views that start one element into their rows (8-byte aligned only), odd K
    w = wl.cpmm_uniform(4200, 50, 101, 40, 50, 1)
    Pfull = _t(np.concatenate([np.zeros((50, 1), dtype=np.int64), w.P], axis=1))  # 50 x 102
    Pview = Pfull[:, 1:]                          # k = 101 (odd), ldp = 102, offset 8 bytes
    assert np.array_equal(Pview.cpu().numpy(), w.P)
    PA, PB = hlb.cp_mm(Pview, _t(w.A), _t(w.B), w.primes, p_absmax=w.p_absmax, form="fp64")
    want = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1])
    w = wl.cpmm_uniform(4201, 50, 100, 40, 50, 1)
    z = np.zeros((50, 1), dtype=np.int64)
    Pfull = _t(np.concatenate([z, w.P, z], axis=1))  # ldp = 102
    Pview = Pfull[:, 1:101]                       # k = 100 even, but base offset 8 bytes
    assert np.array_equal(Pview.cpu().numpy(), w.P)
    PA, PB = hlb.cp_mm(Pview, _t(w.A), _t(w.B), w.primes, p_absmax=w.p_absmax, form="fp64")
    want = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1])


def test_fp64_trunc_both_paths_exact_regime():
    # Strategy 2 in its exact regime (no partial sum reaches 2^53): both paths are bit-exact
    g = wl.rng(4300)
    q = (1 << 31) - 1
    m, k, n = 70, 98, 90
    P = g.integers(-(1 << 15), 1 << 15, size=(m, k))
    A = g.integers(0, q, size=(1, k, n), dtype=np.uint64)
    B = g.integers(0, q, size=(1, k, n), dtype=np.uint64)
    want = oracle.cp_mm(P, A, B, [q])
    got = _both_paths(lambda: tuple(_np(x) for x in hlb.cp_mm_trunc_b(_t(P), _t(A), _t(B), [q], 0.0,
                                                                       p_absmax=1 << 15, form="fp64")))
    for gg in got:
        assert np.array_equal(gg[0], want[0]) and np.array_equal(gg[1], want[1])
