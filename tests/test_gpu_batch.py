"""GPU tests of the batched CP-MM: persistent kernel + HIP graph replay + tile classes.

Every product of a batch must be bit-identical to the oracle and to a single hlb_cp_mm of
the same problem; graph replays must track in-place input changes; eager and graph modes
and both tile classes must agree."""
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


def _problems(seed, shapes, primes):
    g = wl.rng(seed)
    out = []
    for (m, k, nA, nB) in shapes:
        P = wl.plaintext_matrix(g, m, k)
        A = np.stack([wl.uniform_residues(g, (k, nA), q) for q in primes]) if nA else np.zeros((len(primes), k, 0), np.uint64)
        B = np.stack([wl.uniform_residues(g, (k, nB), q) for q in primes]) if nB else np.zeros((len(primes), k, 0), np.uint64)
        out.append(dict(P=P, A=A, B=B))
    return out


SHAPES = [(64, 130, 128, 128), (200, 64, 70, 33), (1, 1, 1, 1), (65, 257, 300, 64), (130, 100, 0, 90),
          (33, 700, 129, 129), (256, 64, 64, 200), (7, 5, 9, 3)]


def _run_batch(probs, primes, form="int8", **kw):
    dev = [dict(P=_t(p["P"]), A=_t(p["A"]), B=_t(p["B"]), p_absmax=kw.get("p_absmax", 1 << 20)) for p in probs]
    outs = hlb.cp_mm_batch(dev, primes, form=form)
    return dev, [(_np(a), _np(b)) for a, b in outs]


@pytest.mark.parametrize("bits", [45, 50])
def test_batch_matches_oracle_and_single_calls(bits):
    primes = wl.ntt_primes(bits, 3)
    probs = _problems(11 + bits, SHAPES, primes)
    _, got = _run_batch(probs, primes)
    for p, (PA, PB) in zip(probs, got):
        wantA, wantB = oracle.cp_mm(p["P"], p["A"], p["B"], primes)
        assert np.array_equal(PA, wantA) and np.array_equal(PB, wantB)
        sA, sB = hlb.cp_mm(_t(p["P"]), _t(p["A"]), _t(p["B"]), primes, p_absmax=1 << 20, form="int8")
        assert np.array_equal(_np(sA), PA) and np.array_equal(_np(sB), PB)


def test_graph_replay_tracks_inputs_and_matches_eager():
    primes = wl.ntt_primes(45, 4)
    shapes = [(96, 200, 160, 160), (64, 64, 64, 64), (150, 333, 70, 70)]
    probs = _problems(21, shapes, primes)
    dev = [dict(P=_t(p["P"]), A=_t(p["A"]), B=_t(p["B"]), p_absmax=1 << 20) for p in probs]
    outs = [(torch.empty((4, s[0], s[2]), dtype=torch.int64, device=DEV),
             torch.empty((4, s[0], s[3]), dtype=torch.int64, device=DEV)) for s in shapes]
    for d, (a, b) in zip(dev, outs):
        d["PA"], d["PB"] = a, b
    g = wl.rng(22)
    for replay in range(4):
        if replay:
            # change every input in place (same pointers, same signature): a replay must see it
            for p, d in zip(probs, dev):
                p["P"] = wl.plaintext_matrix(g, *p["P"].shape)
                p["A"] = np.stack([wl.uniform_residues(g, p["A"].shape[1:], q) for q in primes])
                d["P"].copy_(_t(p["P"]))
                d["A"].copy_(_t(p["A"]))
            torch.cuda.synchronize()
        hlb.cp_mm_batch(dev, primes, form="int8")
        # eager work between replays
        _ = (dev[0]["P"] * 3).sum().item()
        for p, (a, b) in zip(probs, outs):
            wantA, wantB = oracle.cp_mm(p["P"], p["A"], p["B"], primes)
            assert np.array_equal(_np(a), wantA) and np.array_equal(_np(b), wantB), replay
    # eager (no graph) mode gives the same bytes
    keep = [(_np(a).copy(), _np(b).copy()) for a, b in outs]
    try:
        hlb.set_option(hlb.OPT_BATCH_GRAPH, 0)
        for a, b in outs:
            a.zero_()
            b.zero_()
        hlb.cp_mm_batch(dev, primes, form="int8")
    finally:
        hlb.set_option(hlb.OPT_BATCH_GRAPH, 1)
    for (a, b), (ka, kb) in zip(outs, keep):
        assert np.array_equal(_np(a), ka) and np.array_equal(_np(b), kb)


@pytest.mark.parametrize("cls", [0, 1])
def test_tile_classes_agree(cls):
    primes = wl.ntt_primes(50, 2)
    probs = _problems(31, SHAPES[:5], primes)
    try:
        hlb.set_option(hlb.OPT_FORCE_CLASS, cls)
        _, got = _run_batch(probs, primes)
        single = [hlb.cp_mm(_t(p["P"]), _t(p["A"]), _t(p["B"]), primes, p_absmax=1 << 20) for p in probs]
        single = [(_np(a), _np(b)) for a, b in single]
    finally:
        hlb.set_option(hlb.OPT_FORCE_CLASS, -1)
    for p, (PA, PB), (sA, sB) in zip(probs, got, single):
        wantA, wantB = oracle.cp_mm(p["P"], p["A"], p["B"], primes)
        assert np.array_equal(PA, wantA) and np.array_equal(PB, wantB)
        assert np.array_equal(sA, wantA) and np.array_equal(sB, wantB)


def test_batch_degenerate_members_and_measured_bound():
    primes = wl.ntt_primes(50, 2)
    shapes = [(40, 0, 8, 8), (0, 10, 5, 5), (30, 70, 0, 0), (50, 90, 40, 40)]
    probs = _problems(41, shapes, primes)
    dev = [dict(P=_t(p["P"]), A=_t(p["A"]), B=_t(p["B"]), p_absmax=0) for p in probs]
    for d, s in zip(dev, shapes):
        d["PA"] = torch.full((2, s[0], s[2]), 5, dtype=torch.int64, device=DEV)
        d["PB"] = torch.full((2, s[0], s[3]), 5, dtype=torch.int64, device=DEV)
    hlb.cp_mm_batch(dev, primes, form="int8")
    assert (_np(dev[0]["PA"]) == 0).all() and (_np(dev[0]["PB"]) == 0).all()  # k = 0 -> zeros
    wantA, wantB = oracle.cp_mm(probs[3]["P"], probs[3]["A"], probs[3]["B"], primes)
    assert np.array_equal(_np(dev[3]["PA"]), wantA) and np.array_equal(_np(dev[3]["PB"]), wantB)


def test_batch_forced_fold_and_fp64_form():
    primes = wl.ntt_primes(50, 2)
    probs = _problems(51, [(70, 600, 65, 65), (33, 300, 100, 20)], primes)
    try:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 128)
        _, got = _run_batch(probs, primes)
    finally:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 0)
    _, got64 = _run_batch(probs, primes, form="fp64")
    for p, (PA, PB), (fA, fB) in zip(probs, got, got64):
        wantA, wantB = oracle.cp_mm(p["P"], p["A"], p["B"], primes)
        assert np.array_equal(PA, wantA) and np.array_equal(PB, wantB)
        assert np.array_equal(fA, wantA) and np.array_equal(fB, wantB)
