"""Synchronous launches: the same seeded calls run in a child process with every kernel launch
and copy serialized by the HIP runtime (AMD_SERIALIZE_KERNEL=3, AMD_SERIALIZE_COPY=3) and in
one without; the outputs must be byte-identical, and equal to the oracle's.  A missing wait or
a launch that depends on a stream-ordering accident would show up as a difference.  Covers
CP-MM in every form and both batch forms (the multimodular batch replayed from its graph)."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import hashlib, json
import numpy as np, torch
import workloads as wl, paper_2503_16080_amd as h
def dig(*ts):
    m = hashlib.sha256()
    for t in ts:
        torch.cuda.synchronize()
        m.update(t.cpu().numpy().tobytes())
    return m.hexdigest()
def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int64) if a.dtype == np.uint64 else a).cuda()
out = {}
w = wl.cpmm_uniform(7300, 300, 700, 260, 50, 3)
P, A, B = dev(w.P), dev(w.A), dev(w.B)
for form in ("int8_crt", "int8", "fp64"):
    PA, PB = h.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form)
    out[form] = dig(PA, PB)
primes = wl.ntt_primes(45, 2)
g = wl.rng(7301)
probs = []
for m, k, n in ((300, 400, 260), (130, 257, 500), (64, 900, 128)):
    probs.append(dict(P=dev(wl.plaintext_matrix(g, m, k)),
                      A=dev(np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])),
                      B=dev(np.stack([wl.uniform_residues(g, (k, n), q) for q in primes])),
                      p_absmax=1 << 20,
                      PA=torch.empty((2, m, n), dtype=torch.int64, device="cuda"),
                      PB=torch.empty((2, m, n), dtype=torch.int64, device="cuda")))
for form in ("int8_crt", "int8"):
    for rep in range(2):
        h.cp_mm_batch(probs, primes, form=form)
        out[f"batch_{form}_{rep}"] = dig(*[t for p in probs for t in (p["PA"], p["PB"])])
print(json.dumps(out))
"""


def _run(serialize):
    env = dict(os.environ)
    for k in ("AMD_SERIALIZE_KERNEL", "AMD_SERIALIZE_COPY"):
        env.pop(k, None)
    if serialize:
        env.update(AMD_SERIALIZE_KERNEL="3", AMD_SERIALIZE_COPY="3")
    print(f"child process, serialized launches: {serialize}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_serialized_launches_give_identical_outputs():
    ser, par = _run(True), _run(False)
    assert ser == par
    w = wl.cpmm_uniform(7300, 300, 700, 260, 50, 3)
    wantA, wantB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
    m = hashlib.sha256()
    m.update(np.ascontiguousarray(wantA).tobytes())
    m.update(np.ascontiguousarray(wantB).tobytes())
    for form in ("int8_crt", "int8", "fp64"):
        assert ser[form] == m.hexdigest(), form
    for form in ("int8_crt", "int8"):
        assert ser[f"batch_{form}_0"] == ser[f"batch_{form}_1"]
    assert ser["batch_int8_crt_0"] == ser["batch_int8_0"]
