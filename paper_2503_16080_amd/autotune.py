"""Tile-class autotuner for the INT8 form.

For each problem shape bucket (ciphertext digit count, floor(log2) of m, n and k), times a
CP-MM of a representative shape with each tile class forced (HIP events around the limb
GEMM inside the library), keeps the faster class, installs it in the library's table
(hlb_tune_set) and optionally writes the table file that HLB_TUNE_CACHE / hlb_tune_load
read back.  Inputs are random residues drawn on the device: only the timing matters here.

Usage: python -m paper_2503_16080_amd.autotune --out tune.txt --shapes 64x1024x1024 ...
(shapes are m x n x k; n is the column count of one output matrix).
"""
from __future__ import annotations

import argparse
import math

import torch

from . import (FORM_INT8, OPT_FORCE_CLASS, OPT_PROFILE, hlb_cp_mm, hlb_plan, load, profile_read,
               profile_reset, set_option)


def _time_class(cls: int, m: int, n: int, k: int, primes, reps: int) -> float:
    dev = torch.device("cuda")
    L = len(primes)
    P = torch.randint(-(1 << 20), (1 << 20) + 1, (m, k), dtype=torch.int64, device=dev)
    A = torch.stack([torch.randint(0, q, (k, n), dtype=torch.int64, device=dev) for q in primes])
    PA = torch.empty((L, m, n), dtype=torch.int64, device=dev)
    PB = torch.empty_like(PA)
    set_option(OPT_FORCE_CLASS, cls)
    try:
        hlb_cp_mm(P, A, A, primes, p_absmax=1 << 20, form=FORM_INT8, out=(PA, PB))
        torch.cuda.synchronize()
        profile_reset()
        set_option(OPT_PROFILE, 1)
        for _ in range(reps):
            hlb_cp_mm(P, A, A, primes, p_absmax=1 << 20, form=FORM_INT8, out=(PA, PB))
        torch.cuda.synchronize()
        set_option(OPT_PROFILE, 0)
        launches, ms = profile_read("gemm_i8")
        profile_reset()
    finally:
        set_option(OPT_FORCE_CLASS, -1)
    return ms / max(launches, 1)


def tune(shapes, primes, reps: int = 3, out_path: str | None = None, verbose: bool = False):
    """Measures both tile classes for every (m, n, k) in `shapes`; returns table entries
    (x_digits, log2m, log2n, log2k, cls, ms0, ms1)."""
    lib = load()
    x_digits = hlb_plan(1, 64, max(primes), 1 << 20, "int8")["x_limbs"]
    entries = []
    for (m, n, k) in shapes:
        t0 = _time_class(0, m, n, k, primes, reps)
        t1 = _time_class(1, m, n, k, primes, reps)
        cls = 0 if t0 <= t1 else 1
        key = (x_digits, int(math.log2(m)), int(math.log2(n)), int(math.log2(k)))
        if lib.hlb_tune_set(*key, cls) != 0:
            raise RuntimeError("hlb_tune_set rejected an entry")
        entries.append((*key, cls, t0, t1))
        if verbose:
            print(f"m={m} n={n} k={k}: class0 {t0:.3f} ms, class1 {t1:.3f} ms -> {cls}", flush=True)
    if out_path:
        with open(out_path, "w") as f:
            f.write("# x_digits log2m log2n log2k class   (written by paper_2503_16080_amd.autotune)\n")
            for e in entries:
                f.write(f"{e[0]} {e[1]} {e[2]} {e[3]} {e[4]}   # {e[5]:.4f} ms vs {e[6]:.4f} ms\n")
    return entries


def _parse_shape(s: str):
    m, n, k = (int(v) for v in s.lower().split("x"))
    return m, n, k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", nargs="+", required=True, help="m x n x k, e.g. 64x1024x1024")
    ap.add_argument("--bits", type=int, default=45)
    ap.add_argument("--primes", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    import workloads
    primes = workloads.ntt_primes(a.bits, a.primes)
    tune([_parse_shape(s) for s in a.shapes], primes, reps=a.reps, out_path=a.out, verbose=True)


if __name__ == "__main__":
    main()
