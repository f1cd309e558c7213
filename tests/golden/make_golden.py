"""Writes the stored expected values under tests/golden/ (calls only the oracle).

Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as wl  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()


def main():
    out = {"note": "expected values written by tests/golden/make_golden.py from the CPU oracle",
           "cases": []}
    # Mod-PP-MM, both operands full residues (uniform in [0, q)), one 50-bit prime.
    for (m, k, n, bits, seed) in [(37, 70, 29, 50, 31), (64, 256, 64, 52, 32)]:
        g = wl.rng(seed)
        q = wl.ntt_primes(bits, 1, skip=seed % 8)[0]
        P = wl.uniform_residues(g, (m, k), q)
        X = wl.uniform_residues(g, (k, n), q)
        C = oracle.mod_pp_mm(q, P, X)
        out["cases"].append(dict(kind="mod_pp_mm", m=m, k=k, n=n, bits=bits, seed=seed, q=q,
                                 sha256=digest(C), corner=[int(C[0, 0]), int(C[-1, -1])]))
    # CP-MM over 3 primes with the 2^20-scaled plaintext.
    for (m, k, n, bits, L, seed) in [(48, 96, 40, 50, 3, 33)]:
        w = wl.cpmm_uniform(seed, m, k, n, bits, L)
        PA, PB = oracle.cp_mm(w.P, w.A, w.B, w.primes)
        out["cases"].append(dict(kind="cp_mm", m=m, k=k, n=n, bits=bits, L=L, seed=seed,
                                 primes=w.primes, sha256_PA=digest(PA), sha256_PB=digest(PB),
                                 corner=[int(PA[0, 0, 0]), int(PB[-1, -1, -1])]))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_regression.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
