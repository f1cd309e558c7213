"""hlb_cp_mm_noalloc, the entry point that allocates nothing (its workspace is the library's
static scratch array), against hlb_cp_mm, the entry point it is a variant of: bit-identical
outputs in every form, on consecutive calls that reuse the array with a smaller second
problem, a clear refusal of problems beyond the array, and a caller's graph capture of the
call (which then records no allocation).  The outputs are also checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_16080_amd as hlb
import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"
FORMS = ["int8_crt", "int8", "fp64"]


def _t(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("form", FORMS)
def test_noalloc_matches_cp_mm_on_consecutive_calls(form):
    # larger problems, then a smaller one over fewer primes: each call reuses the array that
    # still holds the last call's planes (the first, with 6 K blocks and 704 tiles, runs the
    # persistent multimodular GEMM, whose queue counters also live in the array)
    for i, (m, k, n, L) in enumerate([(1024, 384, 1024, 3), (700, 900, 520, 3), (130, 257, 75, 2)]):
        print(f"\n[noalloc] form={form} call {i}: m={m} k={k} n={n} L={L}", flush=True)
        w = wl.cpmm_uniform(9300 + i, m, k, n, 50, L)
        P, A, B = _t(w.P), _t(w.A), _t(w.B)
        refA, refB = hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form)
        PA = torch.full((L, m, n), -1, dtype=torch.int64, device=DEV)
        PB = torch.full((L, m, n), -1, dtype=torch.int64, device=DEV)
        hlb.cp_mm_noalloc(P, A, B, w.primes, w.p_absmax, form=form, out=(PA, PB))
        gotA, gotB = _np(PA), _np(PB)
        assert np.array_equal(gotA, _np(refA)) and np.array_equal(gotB, _np(refB)), (form, i)
        wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
        assert np.array_equal(gotA, wantA) and np.array_equal(gotB, wantB), (form, i)


def test_noalloc_refuses_what_does_not_fit_and_a_measured_bound():
    # multimodular workspace of d = 2048 over 3 primes: 6 x 2048 x 2048 x 11 residue bytes of
    # the ciphertext alone, above the 256 MiB array -> HLB_ESCRATCH, outputs untouched
    d, L = 2048, 3
    primes, P, A, B = wl.cpmm_uniform_device(9400, d, d, d, 50, L)
    PA = torch.full((L, d, d), 5, dtype=torch.int64, device=DEV)
    PB = torch.full((L, d, d), 5, dtype=torch.int64, device=DEV)
    torch.cuda.synchronize()
    with pytest.raises(hlb.HlbError) as e:
        hlb.cp_mm_noalloc(P, A, B, primes, 1 << 20, form="int8_crt", out=(PA, PB))
    assert e.value.status == 7
    assert "scratch" in hlb.hlb_status_str(7)
    torch.cuda.synchronize()
    assert bool((PA == 5).all()) and bool((PB == 5).all())
    with pytest.raises(hlb.HlbError) as e:
        hlb.cp_mm_noalloc(P[:64, :64], A[:, :64, :64].contiguous(), B[:, :64, :64].contiguous(), primes, 0,
                          form="int8_crt")
    assert e.value.status == 1


@pytest.mark.parametrize("form", FORMS)
def test_noalloc_under_caller_graph_capture(form):
    w = wl.cpmm_uniform(9500, 300, 700, 260, 50, 2)
    want = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    PA = torch.empty((2, 300, 260), dtype=torch.int64, device=DEV)
    PB = torch.empty_like(PA)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        hlb.cp_mm_noalloc(P, A, B, w.primes, w.p_absmax, form=form, out=(PA, PB), stream=s)
    for rep in range(3):
        PA.fill_(7)
        PB.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1]), (form, rep)
        # eager use of the same array between replays (a different, smaller problem)
        v = wl.cpmm_uniform(9600 + rep, 64, 96, 40, 50, 1)
        vA, vB = hlb.cp_mm_noalloc(_t(v.P), _t(v.A), _t(v.B), v.primes, v.p_absmax, form=form)
        wv = oracle.cp_mm(v.P, v.A, v.B, v.primes)
        assert np.array_equal(_np(vA), wv[0]) and np.array_equal(_np(vB), wv[1]), (form, rep, "eager")
