"""The library's per-stream workspace block: calls of alternating shapes and forms reuse and
grow one block per stream, two streams keep separate blocks, hlb_release returns them, and a
caller can capture a call in a graph (its workspace then belongs to the graph).  Every result
is checked bit for bit against the oracle (the plain definition of CP-MM)."""
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


# (m, k, n, L): small, large, small again, so the block grows and is then reused
SHAPES = [(40, 70, 33, 2), (300, 1100, 520, 3), (64, 200, 64, 1), (513, 260, 300, 2), (33, 65, 17, 1)]
FORMS = ["int8_crt", "int8", "fp64"]


def _case(i, shape):
    m, k, n, L = shape
    w = wl.cpmm_uniform(7100 + i, m, k, n, 50, L)
    want = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    return w, want


def test_alternating_shapes_and_forms_on_one_stream():
    cases = [_case(i, s) for i, s in enumerate(SHAPES)]
    for rep in range(2):
        for i, (w, want) in enumerate(cases):
            form = FORMS[(i + rep) % len(FORMS)]
            PA, PB = hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes, p_absmax=w.p_absmax, form=form)
            assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1]), (rep, i, form)


def test_two_streams_without_host_sync_between_calls():
    cases = [_case(20 + i, s) for i, s in enumerate(SHAPES[:4])]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    inputs = [(_t(w.P), _t(w.A), _t(w.B)) for w, _ in cases]
    torch.cuda.synchronize()
    outs = []
    for i, ((w, _), (P, A, B)) in enumerate(zip(cases, inputs)):
        st = streams[i % 2]
        with torch.cuda.stream(st):
            outs.append(hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=FORMS[i % 2], stream=st))
    torch.cuda.synchronize()
    for (w, want), (PA, PB) in zip(cases, outs):
        assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1])


def test_release_between_calls():
    w, want = _case(40, SHAPES[1])
    for _ in range(2):
        PA, PB = hlb.cp_mm(_t(w.P), _t(w.A), _t(w.B), w.primes, p_absmax=w.p_absmax, form="int8_crt")
        assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1])
        hlb.release()


# (300, 700, 260, 2): 11 K blocks, one GEMM workgroup per tile; (600, 640, 700, 2): 10 K
# blocks and 264 tiles, the persistent multimodular launch (a queue-counter fill kernel, then
# workgroups taking several tiles each)
@pytest.mark.parametrize("form,shape", [(f, (300, 700, 260, 2)) for f in FORMS] + [("int8_crt", (600, 640, 700, 2))])
def test_caller_captures_cp_mm_in_a_graph(form, shape):
    # under capture the workspace is a graph-owned allocation; every replay, with eager work
    # and synchronisations between replays, matches the oracle
    m, k, n, L = shape
    w, want = _case(60, shape)
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    PA = torch.empty((L, m, n), dtype=torch.int64, device=DEV)
    PB = torch.empty_like(PA)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form, out=(PA, PB), stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form, out=(PA, PB), stream=s)
    for _ in range(3):
        PA.fill_(7)
        PB.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1])
        torch.randn(1000, device=DEV).sum().item()


def test_capture_with_measured_bound_is_refused_before_any_enqueue():
    # p_absmax = 0 asks the library to measure max |P| on the device, which needs a copy to the
    # host and a synchronization: on a capturing stream the call must fail with HLB_EINVAL
    # before it enqueues anything, leaving the capture intact (the graph then holds only the
    # caller's own work and replays it).
    w, want = _case(61, (120, 300, 96, 2))
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    PA = torch.empty((2, 120, 96), dtype=torch.int64, device=DEV)
    PB = torch.empty_like(PA)
    flag = torch.zeros(4, dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    status = {}
    with torch.cuda.graph(g, stream=s):
        flag.add_(1)
        for name, fn in (("cp_mm", lambda: hlb.cp_mm(P, A, B, w.primes, p_absmax=0, form="int8_crt",
                                                       out=(PA, PB), stream=s)),
                         ("absmax", lambda: hlb.plaintext_absmax(P, stream=s)),
                         ("validate", lambda: hlb.validate_residues(A[0], w.primes[0], stream=s)),
                         ("batch", lambda: hlb.cp_mm_batch([dict(P=P, A=A, B=B, p_absmax=0, PA=PA, PB=PB)],
                                                           w.primes, form="int8_crt", stream=s))):
            try:
                fn()
                status[name] = 0
            except hlb.HlbError as e:
                status[name] = e.status
        flag.add_(1)
    assert status == {"cp_mm": 1, "absmax": 1, "validate": 1, "batch": 1}, status
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert flag.tolist() == [2 * (rep + 1)] * 4
    # the same call outside capture measures the bound and is exact
    PA2, PB2 = hlb.cp_mm(P, A, B, w.primes, p_absmax=0, form="int8_crt")
    assert np.array_equal(_np(PA2), want[0]) and np.array_equal(_np(PB2), want[1])


def test_many_short_lived_streams_reuse_and_evict_blocks():
    # torch hands out pooled stream handles round-robin, so the calls below reuse handles of
    # streams whose Python objects are gone, and touch more streams than the library keeps
    # workspace blocks for (older blocks are freed after their last use): nothing is
    # synchronised on the host until the end, and every result must match the oracle.
    cases = [_case(90 + i, s) for i, s in enumerate(SHAPES)]
    torch.cuda.synchronize()
    pending = []
    for rep in range(3):
        for i, (w, want) in enumerate(cases):
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                P, A, B = _t(w.P), _t(w.A), _t(w.B)
                out = hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=FORMS[(i + rep) % 3], stream=st)
            pending.append((rep, i, want, out))
    torch.cuda.synchronize()
    for rep, i, want, (PA, PB) in pending:
        assert np.array_equal(_np(PA), want[0]) and np.array_equal(_np(PB), want[1]), (rep, i)
