"""GPU failure paths forced from the host: a workspace cap makes every form's allocation
fail with HLB_ENOMEM before any kernel touches the outputs, and the next uncapped call is
exact again (against the oracle)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_16080_amd as hlb
import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"
ENOMEM = 4


def _t(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("form", ["int8_crt", "int8", "fp64"])
def test_workspace_cap_fails_cleanly_then_recovers(form):
    w = wl.cpmm_uniform(6100, 512, 512, 512, 50, 2)
    P, A, B = _t(w.P), _t(w.A), _t(w.B)
    PA = torch.full((2, 512, 512), -1, dtype=torch.int64, device=DEV)
    PB = torch.full((2, 512, 512), -1, dtype=torch.int64, device=DEV)
    try:
        hlb.set_option(hlb.OPT_WS_CAP, 1 << 20)
        with pytest.raises(hlb.HlbError) as err:
            hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form, out=(PA, PB))
        assert err.value.status == ENOMEM
        assert bool((PA == -1).all()) and bool((PB == -1).all())
    finally:
        hlb.set_option(hlb.OPT_WS_CAP, 0)
    hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form, out=(PA, PB))
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    assert np.array_equal(_np(PA), wantA) and np.array_equal(_np(PB), wantB)


@pytest.mark.parametrize("form", ["int8", "int8_crt"])
def test_eager_batch_workspace_cap(form):
    primes = wl.ntt_primes(45, 2)
    g = wl.rng(6200)
    probs, want = [], []
    for m, k, n in ((300, 400, 260), (130, 257, 500)):
        P = wl.plaintext_matrix(g, m, k)
        A = np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])
        B = np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])
        probs.append(dict(P=_t(P), A=_t(A), B=_t(B), p_absmax=1 << 20,
                          PA=torch.full((2, m, n), -1, dtype=torch.int64, device=DEV),
                          PB=torch.full((2, m, n), -1, dtype=torch.int64, device=DEV)))
        want.append(oracle.cp_mm(P, A, B, primes))
    hlb.set_option(hlb.OPT_BATCH_GRAPH, 0)
    try:
        hlb.set_option(hlb.OPT_WS_CAP, 1 << 20)
        with pytest.raises(hlb.HlbError) as err:
            hlb.cp_mm_batch(probs, primes, form=form)
        assert err.value.status == ENOMEM
        for p in probs:
            assert bool((p["PA"] == -1).all()) and bool((p["PB"] == -1).all())
        hlb.set_option(hlb.OPT_WS_CAP, 0)
        hlb.cp_mm_batch(probs, primes, form=form)
    finally:
        hlb.set_option(hlb.OPT_WS_CAP, 0)
        hlb.set_option(hlb.OPT_BATCH_GRAPH, 1)
    for p, (wA, wB) in zip(probs, want):
        assert np.array_equal(_np(p["PA"]), wA) and np.array_equal(_np(p["PB"]), wB)


def test_digit_form_refuses_k_beyond_32_bit_panel_offsets():
    """The digit tiles address their K panels with 32-bit byte offsets: a K whose panel would
    pass 2^32 bytes is refused with HLB_EINVAL before anything runs, and the output is left
    untouched; the multimodular form refuses k > 131071 with HLB_EBOUND."""
    q = wl.ntt_primes(50, 1)[0]
    k = 10_000_000
    print(f"\n[failures] digit form k={k}", flush=True)
    P = torch.ones((1, k), dtype=torch.int64, device=DEV)
    X = torch.ones((k, 1), dtype=torch.int64, device=DEV)
    C = torch.full((1, 1), -1, dtype=torch.int64, device=DEV)
    with pytest.raises(hlb.HlbError) as err:
        hlb.mod_pp_mm(q, P, X, form="int8", out=C)
    assert err.value.status == 1  # HLB_EINVAL
    with pytest.raises(hlb.HlbError) as err:
        hlb.mod_pp_mm(q, P, X, form="int8_crt", out=C)
    assert err.value.status == 3  # HLB_EBOUND
    assert int(C[0, 0]) == -1
    # a K just inside the digit bound still runs (ones: the product is k mod q)
    k2 = 1 << 20
    got = hlb.mod_pp_mm(q, P[:, :k2].contiguous(), X[:k2].contiguous(), form="int8")
    assert int(_np(got)[0, 0]) == k2 % q


def test_workspace_cap_from_environment():
    """HLB_WS_CAP sets the workspace cap at process start (read once, so each setting runs in
    a child process): a cap of 64 KiB refuses the call with HLB_ENOMEM and leaves the outputs
    untouched; hlb_set_option then lifts it and the same call matches the oracle.  A value
    that is not a positive integer sets no cap."""
    import json
    import os
    import subprocess
    import sys
    code = (
        "import json, numpy as np, torch, oracle, workloads as wl, paper_2503_16080_amd as h\n"
        "w = wl.cpmm_uniform(6101, 300, 260, 200, 50, 2)\n"
        "t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64) if a.dtype == np.uint64 "
        "else np.ascontiguousarray(a)).to('cuda')\n"
        "P, A, B = t(w.P), t(w.A), t(w.B)\n"
        "PA = torch.full((2, 300, 200), -1, dtype=torch.int64, device='cuda'); PB = PA.clone()\n"
        "res = []\n"
        "try:\n"
        "    h.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form='int8_crt', out=(PA, PB)); res.append(0)\n"
        "except h.HlbError as e:\n"
        "    res.append(e.status)\n"
        "torch.cuda.synchronize(); res.append(bool((PA == -1).all()) and bool((PB == -1).all()))\n"
        "h.set_option(h.OPT_WS_CAP, 0)\n"
        "h.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form='int8_crt', out=(PA, PB))\n"
        "wA, wB = oracle.cp_mm(w.P, w.A, w.B, w.primes)\n"
        "res.append(bool(np.array_equal(PA.cpu().numpy().view(np.uint64), wA) and "
        "np.array_equal(PB.cpu().numpy().view(np.uint64), wB)))\n"
        "print(json.dumps(res))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    got = {}
    for cap in ("65536", "12x"):
        env = dict(os.environ, HLB_WS_CAP=cap)
        print(f"child process with HLB_WS_CAP={cap}", flush=True)
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                           timeout=180)
        assert r.returncode == 0, r.stderr[-2000:]
        got[cap] = json.loads(r.stdout.strip().splitlines()[-1])
    assert got["65536"] == [ENOMEM, True, True]
    assert got["12x"] == [0, False, True]
