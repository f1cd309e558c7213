"""HLB_OPT_VALIDATE: with the option on, hlb_mod_pp_mm, hlb_cp_mm and hlb_cp_mm_batch check
their inputs on the device first -- every residue below its modulus, every |P| within the
stated p_absmax -- and refuse a violation with HLB_ERANGE before writing any output; inputs in
range give the oracle's result as without the checks.  The checks synchronise the stream, so
on a capturing stream the call is refused with HLB_EINVAL before it enqueues anything."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_16080_amd as hlb
import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"
EINVAL, ERANGE = 1, 2


def _t(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture
def validate():
    hlb.set_option(hlb.OPT_VALIDATE, 1)
    yield
    hlb.set_option(hlb.OPT_VALIDATE, 0)


def _refused(fn, status, *untouched):
    with pytest.raises(hlb.HlbError) as err:
        fn()
    assert err.value.status == status
    torch.cuda.synchronize()
    for t in untouched:
        assert bool((t == -1).all())


@pytest.mark.parametrize("form", ["int8_crt", "int8", "fp64"])
def test_validate_cp_mm(validate, form):
    print(f"\n[validate] cp_mm form={form}", flush=True)
    m, k, n, L = 70, 130, 50, 2
    w = wl.cpmm_uniform(6200, m, k, n, 50, L)
    want = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    PA = torch.full((L, m, n), -1, dtype=torch.int64, device=DEV)
    PB = torch.full_like(PA, -1)
    call = lambda P_, A_, B_: hlb.cp_mm(P_, A_, B_, w.primes, p_absmax=w.p_absmax, form=form, out=(PA, PB))
    bad = A.clone()
    bad[1, 77, 13] = w.primes[1]  # a residue equal to its prime
    _refused(lambda: call(P, A, bad), ERANGE, PA, PB)
    _refused(lambda: call(P, bad, B), ERANGE, PA, PB)
    for v in (w.p_absmax + 1, -(w.p_absmax + 1)):  # a plaintext entry past its bound
        Pbad = P.clone()
        Pbad[5, 9] = v
        _refused(lambda: call(Pbad, A, B), ERANGE, PA, PB)
    call(P, A, B)
    assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1])


def test_validate_mod_pp_mm_and_batch(validate):
    print("\n[validate] mod_pp_mm and batch", flush=True)
    w = wl.cpmm_uniform(6201, 40, 90, 60, 50, 2)
    q = w.primes[0]
    Pq = oracle.residues_of_signed(w.P, q)
    C = torch.full((40, 60), -1, dtype=torch.int64, device=DEV)
    Xbad = _t(w.A[0])
    Xbad[3, 4] = q + 5
    _refused(lambda: hlb.mod_pp_mm(q, _t(Pq), Xbad, out=C), ERANGE, C)
    Pbad = _t(Pq)
    Pbad[0, 0] = q
    _refused(lambda: hlb.mod_pp_mm(q, Pbad, _t(w.A[0]), out=C), ERANGE, C)
    hlb.mod_pp_mm(q, _t(Pq), _t(w.A[0]), out=C)
    assert np.array_equal(_np(C), oracle.mod_pp_mm(q, Pq, w.A[0]))
    # a batch with one bad problem writes nothing
    probs = []
    for j in range(3):
        wj = wl.cpmm_uniform(6210 + j, 50 + 10 * j, 70, 40, 50, 2) if j else w
        probs.append(dict(P=_t(wj.P), A=_t(wj.A), B=_t(wj.B), p_absmax=w.p_absmax,
                          PA=torch.full((2, wj.P.shape[0], wj.A.shape[2]), -1, dtype=torch.int64, device=DEV),
                          PB=torch.full((2, wj.P.shape[0], wj.B.shape[2]), -1, dtype=torch.int64, device=DEV)))
    probs[2]["B"][0, 1, 2] = w.primes[0] + 1
    outs = [t for p in probs for t in (p["PA"], p["PB"])]
    for form in ("int8_crt", "int8"):
        _refused(lambda: hlb.cp_mm_batch(probs, w.primes, form=form), ERANGE, *outs)


def test_validate_on_a_capturing_stream_is_refused(validate):
    print("\n[validate] capture", flush=True)
    w = wl.cpmm_uniform(6220, 60, 80, 40, 50, 2)
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    PA = torch.empty((2, 60, 40), dtype=torch.int64, device=DEV)
    PB = torch.empty_like(PA)
    flag = torch.zeros(4, dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    status = None
    with torch.cuda.graph(g, stream=s):
        flag.add_(1)
        try:
            hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form="int8_crt", out=(PA, PB), stream=s)
            status = 0
        except hlb.HlbError as e:
            status = e.status
        flag.add_(1)
    assert status == EINVAL
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        assert flag.tolist() == [2 * (rep + 1)] * 4
