"""Tile-class autotuner for the INT8 forms.

For each problem shape bucket (floor(log2) of m, n and k, with the ciphertext digit count of
the digit form or the moduli count of the multimodular form), times a CP-MM of a
representative shape with each tile class forced (HIP events around the GEMM inside the
library), keeps the fastest class, installs it in the library's table (hlb_tune_set /
hlb_tune_set_crt) and optionally writes the table file that HLB_TUNE_CACHE / hlb_tune_load
read back.  The multimodular form is timed as a one-problem batch, so that the GEMM timed is
the batch GEMM whose tiles the table then picks (a batch of copies of the shape, enough to
fill the GPU).  Inputs are random residues drawn on the
device: only the timing matters here.

Usage: python -m paper_2503_16080_amd.autotune --out tune.txt --shapes 64x1024x1024 ...
       python -m paper_2503_16080_amd.autotune --form int8_crt --batch-workload --out tune.txt
(shapes are m x n x k; n is the column count of one output matrix; --batch-workload takes
one representative shape per bucket of the 64-problem batch workload).
"""
from __future__ import annotations

import argparse
import math

import torch

from . import (FORM_INT8, OPT_BATCH_GRAPH, OPT_CRT_WIDE, OPT_FORCE_CLASS, OPT_PROFILE, cp_mm_batch, hlb_cp_mm,
               hlb_plan, load, profile_read, profile_reset, set_option)


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


CRT_CLASSES = (0, 1, 2)  # 256 x 128, 256 x 256, 256 x 384 output tiles


def _time_crt_class(cls: int, m: int, n: int, k: int, primes, reps: int, moduli: int) -> float:
    """GEMM time of a multimodular batch of copies of one m x k by k x n problem (both parts n
    wide) with tile class `cls` forced, launched eagerly.  Enough copies to give every CU
    several 256 x 384 tiles, so that the timing is that of a full GPU, as in a batch: a lone
    small problem would only measure how many CUs its tiles reach."""
    dev = torch.device("cuda")
    L = len(primes)
    items = moduli * math.ceil(m / 256) * math.ceil(2 * L * math.ceil(n / 128) / 3)
    copies = max(1, min(64, math.ceil(4096 / items)))
    P = torch.randint(-(1 << 20), (1 << 20) + 1, (m, k), dtype=torch.int64, device=dev)
    A = torch.stack([torch.randint(0, q, (k, n), dtype=torch.int64, device=dev) for q in primes])
    probs = [{"P": P, "A": A, "B": A, "p_absmax": 1 << 20,
              "PA": torch.empty((L, m, n), dtype=torch.int64, device=dev),
              "PB": torch.empty((L, m, n), dtype=torch.int64, device=dev)} for _ in range(copies)]
    set_option(OPT_CRT_WIDE, cls)
    set_option(OPT_BATCH_GRAPH, 0)
    try:
        cp_mm_batch(probs, primes, form="int8_crt")
        torch.cuda.synchronize()
        profile_reset()
        set_option(OPT_PROFILE, 1)
        for _ in range(reps):
            cp_mm_batch(probs, primes, form="int8_crt")
        torch.cuda.synchronize()
        set_option(OPT_PROFILE, 0)
        launches, ms = profile_read("crt_gemm_batch")
        profile_reset()
    finally:
        set_option(OPT_CRT_WIDE, -1)
        set_option(OPT_BATCH_GRAPH, 1)
    return ms / max(launches, 1)


def tune_crt(shapes, primes, reps: int = 3, out_path: str | None = None, verbose: bool = False,
             one_batch: bool = False, margin: float = 0.03):
    """Measures every multimodular tile class for every (m, n, k) in `shapes`; returns table
    entries (moduli, log2m, log2n, log2k, cls, ms per class).  With one_batch the entries are
    keyed by the moduli count of a batch holding all the shapes (a batch plans its moduli for
    its deepest problem), else by each shape's own.  A class other than the widest (2) is
    kept only when it is faster by more than `margin`: a batch runs one GEMM launch per class
    present, and each launch adds its own tail."""
    lib = load()
    entries = []
    kmax = max(k for (_, _, k) in shapes)
    for (m, n, k) in shapes:
        moduli = hlb_plan(1, kmax if one_batch else k, max(primes), 1 << 20, "int8_crt")["p_limbs"]
        times = [_time_crt_class(c, m, n, k, primes, reps, moduli) for c in CRT_CLASSES]
        cls = CRT_CLASSES[min(range(len(times)), key=lambda i: times[i])]
        if times[CRT_CLASSES.index(cls)] > times[CRT_CLASSES.index(2)] * (1.0 - margin):
            cls = 2
        key = (moduli, int(math.log2(m)), int(math.log2(n)), int(math.log2(k)))
        if lib.hlb_tune_set_crt(*key, cls) != 0:
            raise RuntimeError("hlb_tune_set_crt rejected an entry")
        entries.append((*key, cls, times))
        if verbose:
            print(f"m={m} n={n} k={k} D={moduli}: " + ", ".join(f"class {c} {t:.3f} ms" for c, t in zip(CRT_CLASSES, times))
                  + f" -> {cls}", flush=True)
    if out_path:
        with open(out_path, "w") as f:
            f.write("# crt moduli log2m log2n log2k class   (written by paper_2503_16080_amd.autotune; "
                    "batch GEMM ms of classes 0, 1, 2)\n")
            for e in entries:
                f.write(f"crt {e[0]} {e[1]} {e[2]} {e[3]} {e[4]}   # " + " ".join(f"{t:.4f}" for t in e[5]) + "\n")
    return entries


def batch_buckets(seed: int = 1004, count: int = 64):
    """One representative (m, n, k) per (log2 m, log2 n, log2 k) bucket of the batch
    workload (n = k = d), the first problem of each bucket."""
    import workloads
    seen, shapes = set(), []
    for m, d in workloads.batch_shapes(seed, count):
        key = (int(math.log2(m)), int(math.log2(d)), int(math.log2(d)))
        if key not in seen:
            seen.add(key)
            shapes.append((m, d, d))
    return shapes


def _parse_shape(s: str):
    m, n, k = (int(v) for v in s.lower().split("x"))
    return m, n, k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", nargs="+", default=[], help="m x n x k, e.g. 64x1024x1024")
    ap.add_argument("--form", choices=["int8", "int8_crt"], default="int8")
    ap.add_argument("--batch-workload", action="store_true",
                    help="add one shape per (log2 m, log2 n, log2 k) bucket of the 64-problem batch")
    ap.add_argument("--bits", type=int, default=45)
    ap.add_argument("--primes", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    import workloads
    primes = workloads.ntt_primes(a.bits, a.primes)
    shapes = [_parse_shape(s) for s in a.shapes] + (batch_buckets() if a.batch_workload else [])
    if not shapes:
        ap.error("no shapes: give --shapes or --batch-workload")
    if a.form == "int8_crt":
        tune_crt(shapes, primes, reps=a.reps, out_path=a.out, verbose=True, one_batch=a.batch_workload)
    else:
        tune(shapes, primes, reps=a.reps, out_path=a.out, verbose=True)


if __name__ == "__main__":
    main()
