"""GPU parity at the benchmark sizes (d = 4096 and d = 8192, 3 primes of 50 bits), in the
launch configuration the benchmark times: sampled output rows against the oracle computed
row by row, and every output checked by Freivalds' test P (X r) = C r (mod q) with random
vectors r (a wrong matrix passes one vector with probability <= 1/q)."""
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


def _check_large(w, PA, PB, rows, vectors=2, seed=0):
    g = np.random.default_rng(seed)
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes, rows=rows)
    for i, q in enumerate(w.primes):
        assert np.array_equal(PA[i][rows], wantA[i][rows]), (i, "A rows")
        assert np.array_equal(PB[i][rows], wantB[i][rows]), (i, "B rows")
        Pq = oracle.residues_of_signed(w.P, q)
        for X, C, nm in ((w.A[i], PA[i], "A"), (w.B[i], PB[i], "B")):
            for _ in range(vectors):
                r = g.integers(0, q, size=X.shape[1], dtype=np.uint64)
                lhs = oracle.matvec_mod(q, Pq, oracle.matvec_mod(q, X, r))
                assert np.array_equal(lhs, oracle.matvec_mod(q, C, r)), (i, nm, "Freivalds")


@pytest.mark.parametrize("d,form", [(4096, "fp64"), (4096, "int8"), (4096, "int8_crt"), (8192, "int8_crt"),
                                    (8192, "int8"), (8192, "fp64")])
def test_cp_mm_benchmark_size(d, form):
    print(f"\n[large] d={d} form={form}", flush=True)
    w = wl.cpmm_uniform(1000 + d, d, d, d, 50, 3)
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    PA, PB = hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form)
    torch.cuda.synchronize()
    PA = PA.cpu().numpy().view(np.uint64)
    PB = PB.cpu().numpy().view(np.uint64)
    del P, A, B
    rows = [0, 1, 127, 128, d // 2 + 3, d - 1]
    _check_large(w, PA, PB, rows, seed=d)
