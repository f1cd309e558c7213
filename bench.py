"""Benchmark of the CP-MM hot path on one MI355X.

Default workload: CP-MM at d = 8192 -- an 8192 x 8192 plaintext P = floor(2^20 U + 1/2)
times a ciphertext whose a- and b-parts are 8192 x 8192 residue matrices, over 3 RNS primes
of 50 bits -- i.e. 2 * L = 6 Mod-PP-MMs of 8192^3 per step, all bit-exact.

The headline is the INT8-limb form in its multimodular variant (Strategy 3): one step is one
``hlb_cp_mm`` call -- residue splits of the plaintext and of the 6 ciphertext matrices, one
GEMM launch over all 11 moduli x 6 products, and one recombination per output matrix.

Also reported: the INT8 digit form (Strategy 1, 3 x 7 digit products), the FP64-limb form,
a same-shape vendor FP64 GEMM (torch float64 matmul, d^3) and the resulting slowdowns, each
GEMM's roofline position (HIP events around its launches, inside the timed region), and the
CPU oracle's rate on a bounded row sample.  The same line carries one key per other workload,
each with its own roofline block: the CP-MM at d = 4096 over 3 primes in the FP64-limb form,
the CP-MM at d = 16384 over 2 primes in the multimodular form, and the batch of 64 uneven
CP-MMs over 4 primes of 45 bits (graph-replayed batch call, against per-product loops).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extra-configs] [--workload cpmm|batch|trunc]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CP-MM mod-q MACs/s at d=8192, INT8-limb vs FP64-limb; ratio to FP64 GEMM"
INT8_PEAK_TOPS = 5000.0     # MI355X dense INT8 matrix peak, 5.0 POP/s
FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 matrix peak


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--d", type=int, default=8192, help="matrix size (default 8192)")
    ap.add_argument("--primes", type=int, default=3)
    ap.add_argument("--bits", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-limb and dgemm legs")
    ap.add_argument("--no-digit", action="store_true", help="skip the digit (Strategy 1) INT8 leg")
    ap.add_argument("--no-batch-loops", action="store_true",
                    help="batch workload: skip the per-product launch loops")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip the legs of the other workloads: d = 4096 FP64 form, d = 16384 over 2 "
                         "primes, and the 64-problem batch")
    ap.add_argument("--config", type=int, choices=[1, 2, 3, 4, 5],
                    help="one configuration alone, as its own JSON line: 1 a single Mod-PP-MM "
                         "256^3 over one 50-bit prime, FP64-limb form; 2 CP-MM d = 4096 over 3 "
                         "primes, FP64-limb form; 3 the headline (d = 8192 over 3 primes, INT8 "
                         "forms beside the FP64 form); 4 the 64-problem batch; 5 CP-MM d = 16384 "
                         "over 2 primes, multimodular INT8 form")
    ap.add_argument("--workload", choices=["cpmm", "batch", "trunc"], default="cpmm",
                    help="cpmm: one CP-MM of size --d (default); batch: 64 CP-MMs of uneven "
                         "shapes over 4 primes of 45 bits; trunc: the CP-MM of size --d with "
                         "the b-part truncated (Strategy 2) next to the exact one")
    ap.add_argument("--b-err-log2", type=float, default=45.0,
                    help="trunc workload: error budget of the FP64 b-part (log2)")
    ap.add_argument("--b-err-log2-int8", type=float, default=36.5,
                    help="trunc workload: error budget of the INT8 b-part (log2); the default drops "
                         "2 digit shifts, the most that keeps the precision within a bit of exact")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the counter summary from two rocprofv3 --pmc output directories "
                         "(FETCH_SIZE run, WRITE_SIZE run) and exit")
    ap.add_argument("--summarize-mfma", metavar="PMC_DIR",
                    help="write the matrix-pipe summary of each GEMM kernel from one rocprofv3 --pmc "
                         "run of SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE and exit")
    ap.add_argument("--hbm-reference", action="store_true",
                    help="print the HBM rates of plain torch kernels (copy, fill, sum of 2 GiB) "
                         "as one JSON line and exit: the practical ceiling of the HBM-bound "
                         "splits and recombinations")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run 3 device-to-device copies of 1 GiB (a reference kernel of "
                         "known traffic for scaling hardware byte counters)")
    return ap.parse_args()


# The paper's own CP-MM timings at the headline size (Table tab:pcmm, d1 = d2 = d3 = 2^13, in
# its shared-a format: the a-part is 2^12 x d2), with the hardware and settings its text names:
# context, not a target (another machine, one modulus, the b-part approximate).
PAPER_FIGURES = {
    "source": "Table tab:pcmm, 2^13 x 2^13 x 2^13 row",
    "hardware": "Intel Xeon Gold 6342 @ 2.80 GHz, single thread; OpenBLAS 0.3.26 dgemm; HEaaN",
    "a_part_s": 19.1, "b_part_s": 13.3, "total_s": 32.4,
    "mod_q_macs": (1 << 12) * (1 << 13) * (1 << 13) + (1 << 39),
    "setting": "one modulus of about 54 bits (no RNS), b-part approximate (Strategy 2), a-part "
               "exact (Strategy 1, 3 FP64 products); average of 10 runs",
}
PAPER_FIGURES["mod_q_mac_per_s"] = PAPER_FIGURES["mod_q_macs"] / PAPER_FIGURES["total_s"]

_CSRC = os.path.join(ROOT, "paper_2503_16080_amd", "csrc")
# Counter summaries per GEMM kernel: the sources whose SHA-256 they are valid for, and the
# kernel-name substring that selects their dispatches.  One file per kernel and workload.
TRAFFIC = {
    # the persistent launch (every benchmark size has an even K-block count of at least four)
    "crt_gemm": {"sources": [os.path.join(_CSRC, f) for f in ("crt_gemm.hip", "crt_tile.hpp", "crt.hpp", "common.hpp")],
                 "match": "crt_gemm_stream_kernel"},
    "gemm_i8": {"sources": [os.path.join(_CSRC, f) for f in ("gemm_i8.hip", "i8_tile.hpp", "common.hpp")],
                "match": "gemm_i8_kernel"},
    "gemm_f64": {"sources": [os.path.join(_CSRC, f) for f in ("gemm_f64_planes.hip", "common.hpp")],
                 "match": "gemm_f64_planes_kernel"},
    "crt_gemm_batch": {"sources": [os.path.join(_CSRC, f)
                                   for f in ("crt_gemm_batch.hip", "crt_tile.hpp", "crt.hpp", "crt_jobs.hpp",
                                             "common.hpp", "batch.hip")],
                       "match": "crt_gemm_batch_kernel"},
}


def traffic_file(kernel, d, L):
    """The counter summary of `kernel` on the CP-MM of size d over L primes (d = "batch64":
    the 64-problem batch)."""
    name = f"{kernel}_traffic.json" if (d, L) == (8192, 3) else f"{kernel}_traffic_d{d}_L{L}.json"
    return os.path.join(ROOT, "profiles", name)


def kernel_source_hash(kernel: str) -> str:
    """SHA-256 over a GEMM kernel's sources: its counter data is valid only for this hash."""
    import hashlib
    h = hashlib.sha256()
    for p in TRAFFIC[kernel]["sources"]:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, d, L):
    """HBM bytes per launch of `kernel` from its committed counter summary, or None when the
    summary is missing, is for another workload, or predates the current kernel source."""
    try:
        with open(traffic_file(kernel, d, L)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash(kernel) or t.get("d") != d or t.get("primes") != L:
        return None
    return t["fetch_kib"] * 1024 * t["fetch_scale"] + t["write_kib"] * 1024 * t["write_scale"]


def mfma_file(kernel, d, L):
    return os.path.join(ROOT, "profiles", f"{kernel}_mfma_d{d}_L{L}.json")


def measured_mfma(kernel, d, L):
    """Matrix-pipe occupancy of `kernel` from its committed counter summary (busy fraction of
    the SIMD cycles and the clock it ran at), or None when missing or stale."""
    try:
        with open(mfma_file(kernel, d, L)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash(kernel) or t.get("d") != d or t.get("primes") != L:
        return None
    return {"busy_frac": t["mfma_busy_frac"], "clock_ghz": t["clock_ghz"]}


def summarize_mfma(pmc_dir, d, L, kernel, simds=1024, xcds=8):
    """Turns one rocprofv3 --pmc run of SQ_VALU_MFMA_BUSY_CYCLES, SQ_BUSY_CYCLES and
    GRBM_GUI_ACTIVE into the matrix-pipe summary of `kernel`: SQ_VALU_MFMA_BUSY_CYCLES counts
    busy cycles summed over all SIMDs, GRBM_GUI_ACTIVE active cycles summed over the XCDs, so
    busy_frac = MFMA cycles / (SIMDs x cycles per XCD) and clock = cycles per XCD / duration."""
    import csv
    import glob
    import statistics
    (name,) = glob.glob(os.path.join(pmc_dir, "*counter_collection.csv"))
    vals, durs = {}, []
    for r in csv.DictReader(open(name)):
        if TRAFFIC[kernel]["match"] not in r["Kernel_Name"]:
            continue
        vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        if r["Counter_Name"] == "GRBM_GUI_ACTIVE":
            durs.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    if "SQ_VALU_MFMA_BUSY_CYCLES" not in vals or "GRBM_GUI_ACTIVE" not in vals:
        return None
    mfma = statistics.mean(vals["SQ_VALU_MFMA_BUSY_CYCLES"])
    cycles = statistics.mean(vals["GRBM_GUI_ACTIVE"]) / xcds
    out = {"kernel": kernel, "kernel_source_sha256": kernel_source_hash(kernel), "d": d, "primes": L,
           "dispatches": len(durs), "SQ_VALU_MFMA_BUSY_CYCLES": mfma,
           "GRBM_GUI_ACTIVE": statistics.mean(vals["GRBM_GUI_ACTIVE"]),
           "SQ_BUSY_CYCLES": statistics.mean(vals.get("SQ_BUSY_CYCLES", [0.0])),
           "duration_s": statistics.mean(durs), "simds": simds, "xcds": xcds,
           "mfma_busy_frac": mfma / (simds * cycles), "clock_ghz": cycles / statistics.mean(durs) / 1e9}
    with open(mfma_file(kernel, d, L), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def summarize_counters(fetch_dir, write_dir, d, L, kernel):
    """Turns two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, each with
    --copy-calibration) into the counter summary of `kernel`: per-dispatch KiB and the scale
    factors that make the 1 GiB calibration copy read and write exactly 1 GiB."""
    import csv
    import glob
    import statistics

    def per_kernel(path, counter):
        (name,) = glob.glob(os.path.join(path, "*counter_collection.csv"))
        rows = list(csv.DictReader(open(name)))
        gemm = [float(r["Counter_Value"]) for r in rows
                if r["Counter_Name"] == counter and TRAFFIC[kernel]["match"] in r["Kernel_Name"]]
        copy = [float(r["Counter_Value"]) for r in rows
                if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
        return (statistics.mean(gemm) if gemm else None), statistics.mean(copy)

    fetch, fcopy = per_kernel(fetch_dir, "FETCH_SIZE")
    write, wcopy = per_kernel(write_dir, "WRITE_SIZE")
    if fetch is None or write is None:
        return None  # the kernel did not run in these traces
    gib_kib = float(1 << 20)
    out = {"kernel": kernel, "kernel_source_sha256": kernel_source_hash(kernel), "d": d, "primes": L,
           "fetch_kib": fetch, "write_kib": write,
           "fetch_scale": gib_kib / fcopy, "write_scale": gib_kib / wcopy,
           "copy_calibration_kib": {"fetch": fcopy, "write": wcopy, "bytes_copied": 1 << 30}}
    with open(traffic_file(kernel, d, L), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def hbm_reference(reps=10):
    """HBM rates of plain torch kernels on 2 GiB tensors, timed with events: a device copy
    (read + write), a fill (write only) and a sum (read only)."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.int64, device="cuda:0")
    y = torch.empty_like(x)
    nbytes = x.numel() * 8

    def ms(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {"tensor_bytes": nbytes}
    for name, fn, moved in (("copy", lambda: y.copy_(x), 2 * nbytes), ("fill", lambda: y.fill_(3), nbytes),
                            ("sum", lambda: x.sum(), nbytes)):
        t = ms(fn)
        out[name] = {"ms": t, "tbs": moved / (t * 1e-3) / 1e12}
    return out


def _time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_model() -> str:
    """The host CPU's model name (lscpu's "Model name", read from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, gpu_out=None, target_s=15.0):
    """The oracle timed on a bounded row sample of the same CP-MM (all primes, both parts).
    With the GPU's output (PA, PB as host uint64 arrays) given, the sampled rows are compared
    with it after the timing: `rows_equal_to_gpu` is whether every one matches."""
    import numpy as np

    import oracle
    m, k, nA, nB, L = w.m, w.k, w.nA, w.nB, len(w.primes)
    per_row = L * k * (nA + nB)
    t0 = time.perf_counter()
    oracle.cp_mm(w.P, w.A, w.B, w.primes, rows=[0])
    t1 = time.perf_counter() - t0
    rows = int(max(1, min(m, target_s / max(t1, 1e-3))))
    sample = list(range(0, m, max(1, m // rows)))[:rows]
    t0 = time.perf_counter()
    oA, oB = oracle.cp_mm(w.P, w.A, w.B, w.primes, rows=sample)
    dt = time.perf_counter() - t0
    res = {"value": len(sample) * per_row / dt, "unit": "mod-q MAC/s",
           "cores": oracle.num_threads(), "cpu_model": cpu_model(), "kind": "oracle",
           "sample": f"{len(sample)} of {m} output rows of the CP-MM (all {L} primes, a- and "
                     f"b-parts), {dt:.1f} s; rate scales linearly with rows"}
    if gpu_out is not None:
        res["rows_equal_to_gpu"] = bool(np.array_equal(oA[:, sample], gpu_out[0][:, sample])
                                        and np.array_equal(oB[:, sample], gpu_out[1][:, sample]))
    return res


def _roofline(kernel, launches, ms, ops_per_step, steps, d, L, peak, unit, op, bound="mfma"):
    """Roofline block of a kernel timed with HIP events on its launch stream: the algorithmic
    work of one launch (the step's work over its launches of the kernel) over the launch's
    average duration, against the type's dense peak; `traffic` is the committed counter
    summary's HBM bytes per launch when it matches the kernel's current sources."""
    per_step = launches / steps
    ops = ops_per_step / per_step
    rate = ops / (ms * 1e-3) / 1e12
    traffic = measured_traffic(kernel, d, L)
    return {"bound": bound, "achieved": rate, "peak": peak, "unit": unit,
            "frac": rate / peak, "traffic": traffic,
            "traffic_gbs": None if traffic is None else traffic / (ms * 1e-3) / 1e9,
            "mfma_counters": measured_mfma(kernel, d, L),
            "kernel": TRAFFIC[kernel]["match"], "avg_launch_ms": ms, "launches": launches,
            "launches_per_step": per_step, "ops_per_launch": ops, "op": op}


def _profiled(fn, names, steps, warmup):
    """Step time of fn with the library's kernels bracketed by HIP events on their launch
    stream; returns (seconds per step, {name: (launches, average ms)})."""
    import paper_2503_16080_amd as hlb
    for _ in range(warmup):
        fn()
    import torch
    torch.cuda.synchronize()
    hlb.profile_reset()
    hlb.set_option(hlb.OPT_PROFILE, 1)
    s = _time_steps(fn, steps, 0)
    hlb.set_option(hlb.OPT_PROFILE, 0)
    prof = {n: hlb.profile_read(n) for n in names}
    hlb.profile_reset()
    return s, {n: (c, t / max(c, 1)) for n, (c, t) in prof.items()}


def batch_leg(steps, warmup, loops=True):
    """64 independent CP-MMs with d log-uniform in [128, 4096], m log-uniform in [64, 4096],
    n = d, over 4 primes of 45 bits (inputs drawn on the device), as one batch call: the
    multimodular form (batched residue splits, one GEMM launch, batched recombination) and the
    digit form (one persistent launch), both graph-replayed, against per-product loops of
    hlb_cp_mm calls.  The GEMM's roofline comes from the same batch launched eagerly (the
    kernels of a replayed graph cannot be bracketed by events)."""
    import torch

    import paper_2503_16080_amd as hlb
    import workloads as wl

    seed, L, bits = 1004, 4, 45
    # the multimodular batch's tile classes, from the autotuner's table for this workload
    tune_table = os.path.join(ROOT, "paper_2503_16080_amd", "tune_crt_batch64_mi355x.txt")
    if os.path.exists(tune_table):
        hlb.hlb_tune_load(tune_table)
    primes, shapes, probs = wl.batch_problems_device(seed, 64, bits, L)
    dev = torch.device("cuda:0")
    macs = 0
    for p, (m, d) in zip(probs, shapes):
        p["PA"] = torch.empty((L, m, d), dtype=torch.int64, device=dev)
        p["PB"] = torch.empty((L, m, d), dtype=torch.int64, device=dev)
        macs += 2 * L * m * d * d

    def batch(form):
        return lambda: hlb.cp_mm_batch(probs, primes, form=form)

    def loop(form):
        def run():
            for p in probs:
                hlb.cp_mm(p["P"], p["A"], p["B"], primes, p_absmax=1 << 20, form=form, out=(p["PA"], p["PB"]))
        return run

    # the per-product loops first, then the eager batches, then the graph-replayed batches:
    # the graphs' own workspace allocations come last, after every stream-ordered one
    lsteps = max(2, steps // 4)
    s_loop_digit = _time_steps(loop("int8"), lsteps, 1) if loops else None
    s_loop_crt = _time_steps(loop("int8_crt"), lsteps, 1) if loops else None
    hlb.set_option(hlb.OPT_BATCH_GRAPH, 0)
    s_crt_eager, kb = _profiled(batch("int8_crt"), ("crt_split_batch", "crt_gemm_batch", "crt_combine_batch"),
                                steps, warmup)
    s_digit_eager = _time_steps(batch("int8"), lsteps, 1)
    hlb.set_option(hlb.OPT_BATCH_GRAPH, 1)
    s_crt = _time_steps(batch("int8_crt"), steps, warmup)
    s_digit = _time_steps(batch("int8"), steps, warmup)
    crt_moduli = hlb.plan(1, max(d for _, d in shapes), max(primes), 1 << 20, "int8_crt")["p_limbs"]
    classes = [hlb.hlb_tune_class_crt(crt_moduli, m, d, d) for m, d in shapes]
    # the batch GEMM per step: one launch per tile class present
    n_g, ms_g = kb["crt_gemm_batch"]
    gemm_step_ms = ms_g * n_g / steps
    out = {
        "value": macs / s_crt, "unit": "mod-q MAC/s", "ms_per_step": s_crt * 1e3,
        "workload": "64 CP-MMs, d log-uniform [128, 4096], m log-uniform [64, 4096], n = d, 4 primes of "
                    "45 bits, multimodular INT8 form, one graph-replayed batch call",
        "moduli": crt_moduli, "mod_q_macs": macs,
        "roofline": _roofline("crt_gemm_batch", steps, gemm_step_ms,
                              2.0 * crt_moduli * macs, steps, "batch64", L, INT8_PEAK_TOPS, "TOP/s",
                              "int8 MAC x 2 (useful products only)"),
        "kernels_ms": {n: v[1] * v[0] / steps for n, v in kb.items()},
        "tile_classes": {"table": os.path.basename(tune_table) if os.path.exists(tune_table) else None,
                         "problems_per_class": {str(c): classes.count(c) for c in sorted(set(classes))},
                         "gemm_launches_per_step": n_g / steps},
        "eager_batch_ms": s_crt_eager * 1e3,
        "digit_form": {"value": macs / s_digit, "ms": s_digit * 1e3, "digits": [3, 6],
                       "eager_ms": s_digit_eager * 1e3},
    }
    if loops:
        out["per_product_loop_ms"] = s_loop_crt * 1e3
        out["batch_vs_loop_speedup"] = s_loop_crt / s_crt
        out["digit_form"]["per_product_loop_ms"] = s_loop_digit * 1e3
        out["digit_form"]["batch_vs_loop_speedup"] = s_loop_digit / s_digit
    del probs
    torch.cuda.empty_cache()
    return out, shapes


def run_batch(args):
    """The batch workload alone, as its own JSON line."""
    res, shapes = batch_leg(args.steps, args.warmup, loops=not args.no_batch_loops)
    print(json.dumps({
        "metric": "batched CP-MM mod-q MACs/s (64 uneven products, 4 RNS primes of 45 bits)",
        "value": res["value"], "unit": "mod-q MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": res["workload"], "moduli": res["moduli"], "mod_q_macs": res["mod_q_macs"],
                   "shapes_mxd": shapes},
        "roofline": res["roofline"],
        **{k: v for k, v in res.items() if k not in ("value", "ms_per_step", "workload", "roofline")},
    }), flush=True)


def _dgemm_ms(d, steps):
    """Same-shape cleartext FP64 GEMM (vendor library through torch): d x d x d."""
    import torch
    dev = torch.device("cuda:0")
    Xf = torch.rand((d, d), dtype=torch.float64, device=dev)
    Yf = torch.rand((d, d), dtype=torch.float64, device=dev)
    Zf = torch.empty((d, d), dtype=torch.float64, device=dev)
    s = _time_steps(lambda: torch.matmul(Xf, Yf, out=Zf), steps, 2)
    del Xf, Yf, Zf
    return s * 1e3


def config2_leg(steps, warmup):
    """CP-MM at d = 4096 over 3 primes of 50 bits in the plain FP64-limb form (the paper's own
    form: one plaintext limb, three 17-bit ciphertext limbs), beside the multimodular INT8
    form on the same inputs (drawn on the device)."""
    import torch

    import paper_2503_16080_amd as hlb
    import workloads as wl

    d, L = 4096, 3
    primes, P, A, B = wl.cpmm_uniform_device(1002, d, d, d, 50, L)
    PA = torch.empty((L, d, d), dtype=torch.int64, device=P.device)
    PB = torch.empty_like(PA)
    macs = 2 * L * d ** 3
    step = lambda form: (lambda: hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form=form, out=(PA, PB)))
    s_f, kf = _profiled(step("fp64"), ("gemm_f64", "prep_p", "prep_x"), steps, warmup)
    s_c = _time_steps(step("int8_crt"), steps, warmup)
    fplan = hlb.plan(1, d, max(primes), 1 << 20, "fp64")
    ms_dg = _dgemm_ms(d, max(3, steps // 2))
    out = {"value": macs / s_f, "unit": "mod-q MAC/s", "ms_per_step": s_f * 1e3,
           "workload": f"cp_mm d={d} over {L} primes of 50 bits, FP64-limb form "
                       f"({fplan['p_limbs']} x {fplan['x_limbs']} limbs of {fplan['limb_bits']} bits)",
           "roofline": _roofline("gemm_f64", kf["gemm_f64"][0], kf["gemm_f64"][1],
                                 2.0 * fplan["p_limbs"] * fplan["x_limbs"] * macs, steps, d, L,
                                 FP64_PEAK_TFLOPS, "TFLOP/s", "fp64 MAC x 2"),
           "kernels_ms": {n: v[1] for n, v in kf.items()},
           "int8_multimodular_ms": s_c * 1e3, "int8_multimodular_value": macs / s_c,
           "fp64_gemm_ms": ms_dg, "slowdown_vs_fp64_gemm": {"fp64_form": s_f * 1e3 / ms_dg,
                                                            "int8_form": s_c * 1e3 / ms_dg}}
    del P, A, B, PA, PB
    torch.cuda.empty_cache()
    return out


def config1_leg(steps, warmup, cpu=True):
    """One Mod-PP-MM_{q; 256,256,256} (Section 5 notation), P and X uniform in [0, q) for one
    50-bit NTT-friendly prime, in the plain FP64-limb form; the oracle computes the same
    product on the host cores."""
    import numpy as np
    import torch

    import paper_2503_16080_amd as hlb
    import workloads as wl

    n = 256
    q = wl.ntt_primes(50, 1)[0]
    g = wl.rng(1001)
    P = g.integers(0, q, size=(n, n), dtype=np.uint64)
    X = g.integers(0, q, size=(n, n), dtype=np.uint64)
    Pd = torch.from_numpy(P.view(np.int64)).cuda()
    Xd = torch.from_numpy(X.view(np.int64)).cuda()
    C = torch.empty((n, n), dtype=torch.int64, device=Pd.device)
    s, kf = _profiled(lambda: hlb.mod_pp_mm(q, Pd, Xd, form="fp64", out=C), ("gemm_f64",), steps, warmup)
    plan = hlb.plan(0, n, q, 1, "fp64")
    macs = n ** 3
    launches, ms = kf["gemm_f64"]
    f_ops = 2.0 * plan["p_limbs"] * plan["x_limbs"] * macs / max(launches / steps, 1e-9)
    rate = f_ops / (ms * 1e-3) / 1e12
    out = {"value": macs / s, "unit": "mod-q MAC/s", "ms_per_step": s * 1e3,
           "workload": f"mod_pp_mm q of 50 bits, {n}x{n} times {n}x{n} residues, FP64-limb form "
                       f"({plan['p_limbs']} x {plan['x_limbs']} limbs of {plan['limb_bits']} bits)",
           "roofline": {"bound": "mfma", "achieved": rate, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": rate / FP64_PEAK_TFLOPS, "traffic": None, "traffic_gbs": None,
                        "kernel": "gemm_f64_kernel", "avg_launch_ms": ms, "launches": launches,
                        "launches_per_step": launches / steps, "ops_per_launch": f_ops, "op": "fp64 MAC x 2",
                        "note": "one 256^3 product: too few output tiles to fill 256 CUs"}}
    if cpu:
        import oracle
        t0 = time.perf_counter()
        want = oracle.mod_pp_mm(q, P, X)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": macs / dt, "unit": "mod-q MAC/s", "cores": oracle.num_threads(),
                               "cpu_model": cpu_model(), "kind": "oracle",
                               "sample": f"the whole {n}^3 product, {dt:.3f} s"}
        torch.cuda.synchronize()
        out["bit_exact"] = {"oracle_equal": bool(np.array_equal(want, C.cpu().numpy().view(np.uint64)))}
    del Pd, Xd, C
    torch.cuda.empty_cache()
    return out


def run_config(args):
    """--config N: one configuration alone, as its own JSON line."""
    c = args.config
    steps, warmup = args.steps, args.warmup
    line = {"n_gpus": 1, "steps": steps, "warmup": warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "data": "synthetic"}
    if c == 1:
        res = config1_leg(steps, warmup, cpu=not args.no_cpu_baseline)
        metric, dtype = "Mod-PP-MM mod-q MACs/s, 256^3, one 50-bit prime, FP64-limb form", "f64"
    elif c == 2:
        res = config2_leg(steps, warmup)
        metric, dtype = "CP-MM mod-q MACs/s at d=4096, FP64-limb form; ratio to FP64 GEMM", "f64"
    else:
        res = config5_leg(steps, warmup)
        metric, dtype = "CP-MM mod-q MACs/s at d=16384, INT8-limb form; ratio to FP64 GEMM", "i8"
    line.update({"metric": metric, "value": res.pop("value"), "unit": res.pop("unit"),
                 "ms_per_step": res.pop("ms_per_step"), "dtype": dtype,
                 "config": {"workload": res.pop("workload"), "config": c}})
    line.update(res)
    print(json.dumps(line), flush=True)


def config5_leg(steps, warmup):
    """CP-MM at d = 16384 over 2 primes of 50 bits (2 GiB per residue matrix) in the
    multimodular INT8 form, inputs drawn on the device, against the same-shape vendor dgemm."""
    import torch

    import paper_2503_16080_amd as hlb
    import workloads as wl

    d, L = 16384, 2
    primes, P, A, B = wl.cpmm_uniform_device(1005, d, d, d, 50, L)
    PA = torch.empty((L, d, d), dtype=torch.int64, device=P.device)
    PB = torch.empty_like(PA)
    macs = 2 * L * d ** 3
    cplan = hlb.plan(1, d, max(primes), 1 << 20, "int8_crt")
    s_c, kc = _profiled(lambda: hlb.cp_mm(P, A, B, primes, p_absmax=1 << 20, form="int8_crt", out=(PA, PB)),
                        ("crt_gemm", "crt_split", "crt_combine"), steps, warmup)
    del P, A, B, PA, PB
    torch.cuda.empty_cache()
    ms_dg = _dgemm_ms(d, max(2, steps // 3))
    return {"value": macs / s_c, "unit": "mod-q MAC/s", "ms_per_step": s_c * 1e3,
            "workload": f"cp_mm d={d} over {L} primes of 50 bits, multimodular INT8 form "
                        f"({cplan['p_limbs']} moduli)",
            "roofline": _roofline("crt_gemm", kc["crt_gemm"][0], kc["crt_gemm"][1], 2.0 * cplan["p_limbs"] * macs,
                                  steps, d, L, INT8_PEAK_TOPS, "TOP/s", "int8 MAC x 2"),
            "kernels_ms": {n: v[1] for n, v in kc.items()},
            "fp64_gemm_ms": ms_dg, "slowdown_vs_fp64_gemm": s_c * 1e3 / ms_dg}


def run_trunc(args):
    """CP-MM with a truncated b-part (Strategy 2 of Section 6.1) against the exact CP-MM, in
    both limb forms, on the default workload's inputs; the FP64 form with truncation is the
    paper's own configuration (3 limb products on the a-part, 1 on the b-part)."""
    import numpy as np
    import torch

    import paper_2503_16080_amd as hlb
    import workloads as wl

    # Strategy 2's error argument is for one modulus (the paper's setting), so one prime
    d, L = args.d, 1
    w = wl.cpmm_uniform(1003, d, d, d, args.bits, L)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev)
    P, A, B = t(w.P), t(w.A), t(w.B)
    PA = torch.empty((L, d, d), dtype=torch.int64, device=dev)
    PB = torch.empty((L, d, d), dtype=torch.int64, device=dev)
    macs = 2 * L * d * d * d
    res = {}
    for form in ("int8", "fp64"):
        budget = args.b_err_log2_int8 if form == "int8" else args.b_err_log2
        steps = args.steps if form == "int8" else max(2, args.steps // 3)
        warm = args.warmup if form == "int8" else 1
        plan = hlb.plan_trunc_b(d, min(w.primes), max(w.primes), w.p_absmax, budget, form)
        exact = lambda: hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form=form, out=(PA, PB))
        trunc = lambda: hlb.cp_mm_trunc_b(P, A, B, w.primes, budget, p_absmax=w.p_absmax, form=form,
                                          out=(PA, PB))
        s_exact = _time_steps(exact, steps, warm)
        hlb.profile_reset()
        hlb.set_option(hlb.OPT_PROFILE, 1)
        s_trunc = _time_steps(trunc, steps, warm)
        hlb.set_option(hlb.OPT_PROFILE, 0)
        kname = "gemm_i8_trunc" if form == "int8" else "gemm_f64_trunc"
        n_k, ms_k = hlb.profile_read(kname)
        hlb.profile_reset()
        res[form] = {"b_err_log2": budget, "exact_ms": s_exact * 1e3, "trunc_ms": s_trunc * 1e3,
                     "trunc_value": macs / s_trunc, "exact_value": macs / s_exact,
                     "b_part_products": plan["products"], "dropped_shifts": plan["dropped_shifts"],
                     "b_err_bound_log2": plan["err_bound_log2"],
                     "b_part_kernel": kname, "b_part_kernel_ms": ms_k / max(n_k, 1)}
    # the exact multimodular CP-MM of the same inputs, for comparison with both truncations
    s_crt = _time_steps(lambda: hlb.cp_mm(P, A, B, w.primes, p_absmax=w.p_absmax, form="int8_crt", out=(PA, PB)),
                        args.steps, args.warmup)
    Xf = torch.rand((d, d), dtype=torch.float64, device=dev)
    Yf = torch.rand((d, d), dtype=torch.float64, device=dev)
    Zf = torch.empty((d, d), dtype=torch.float64, device=dev)
    s_dgemm = _time_steps(lambda: torch.matmul(Xf, Yf, out=Zf), max(3, args.steps // 2), 2)
    for form in res:
        res[form]["slowdown_vs_fp64_gemm"] = res[form]["trunc_ms"] / (s_dgemm * 1e3)
    del Xf, Yf, Zf, P, A, B, PA, PB
    precision = trunc_precision(d, w.primes[0], args.b_err_log2,
                                sorted({args.b_err_log2, args.b_err_log2_int8, 28.0}, reverse=True))
    print(json.dumps({
        "metric": f"CP-MM mod-q MACs/s at d={d} with the b-part truncated (Strategy 2)",
        "value": res["int8"]["trunc_value"], "unit": "mod-q MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["int8"]["trunc_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": f"cp_mm d={d} over one modulus of {args.bits} bits, a-part exact, "
                               f"b-part error <= 2^{args.b_err_log2_int8:g} (INT8), "
                               f"2^{args.b_err_log2:g} (FP64)"},
        "forms": res, "multimodular_exact_ms": s_crt * 1e3, "fp64_gemm_ms": s_dgemm * 1e3,
        "precision_bits": precision,
    }), flush=True)


def trunc_precision(d, q, budget_fp64, budgets_int8):
    """The paper's precision metric (Section 6: -log2 of the largest entry error of the
    decrypted, decoded product against the cleartext product U M) for the exact CP-MM and
    the truncated b-parts, on a real encryption under one modulus q built on the GPU:
    B = -A S + round(2^15 M) + E, P = round(2^20 U), M and U uniform in [-1, 1], S ternary,
    E rounded Gaussian (sigma 3.2).  |P (round(2^15 M) + E)| stays below q/2, so the centred
    decryption needs no wrap."""
    import torch

    import paper_2503_16080_amd as hlb

    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2025)
    dm, dp = 15, 20
    M = torch.rand((d, d), dtype=torch.float64, device=dev, generator=g) * 2 - 1
    U = torch.rand((d, d), dtype=torch.float64, device=dev, generator=g) * 2 - 1
    S = torch.randint(-1, 2, (d, d), dtype=torch.int64, device=dev, generator=g)
    E = torch.floor(torch.randn((d, d), dtype=torch.float64, device=dev, generator=g) * 3.2 + 0.5).to(torch.int64)
    A = torch.randint(0, q, (1, d, d), dtype=torch.int64, device=dev, generator=g)
    P = torch.floor(U * 2.0 ** dp + 0.5).to(torch.int64)
    B = hlb.hlb_test_encrypt(A, S, hlb.hlb_test_encode(M, 2.0 ** dm) + E, [q])
    want = torch.matmul(U, M)

    def bits(PA, PB):
        D = hlb.hlb_test_decrypt(PA, PB, S, [q])[0]
        Dc = torch.where(D > q // 2, D - q, D).to(torch.float64) / 2.0 ** (dm + dp)
        return float(-torch.log2((Dc - want).abs().max()))

    out = {"exact": bits(*hlb.cp_mm(P, A, B, [q], p_absmax=1 << dp, form="auto"))}
    for form, budgets in (("fp64", (budget_fp64,)), ("int8", budgets_int8)):
        for b in budgets:
            plan = hlb.plan_trunc_b(d, q, q, 1 << dp, b, form)
            key = f"{form}_b{b:g}" + (f"_drop{plan['dropped_shifts']}" if form == "int8" else "")
            out[key] = bits(*hlb.cp_mm_trunc_b(P, A, B, [q], b, p_absmax=1 << dp, form=form))
    return out


def main():
    args = _parse()
    if args.summarize_counters:
        tag = "batch64" if args.workload == "batch" else args.d
        L = 4 if args.workload == "batch" else args.primes
        for kernel in TRAFFIC:
            out = summarize_counters(*args.summarize_counters, tag, L, kernel)
            if out is not None:
                print(json.dumps(out))
        return
    if args.summarize_mfma:
        tag = "batch64" if args.workload == "batch" else args.d
        L = 4 if args.workload == "batch" else args.primes
        for kernel in TRAFFIC:
            out = summarize_mfma(args.summarize_mfma, tag, L, kernel)
            if out is not None:
                print(json.dumps(out))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the CP-MM path has no multi-GPU leg); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2503_16080_amd as hlb
    import workloads as wl

    if args.hbm_reference:
        print(json.dumps(hbm_reference()), flush=True)
        return

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.int64, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.config in (1, 2, 5):
        run_config(args)
        return
    if args.config == 3:
        args.no_extra_configs = True
    if args.workload == "batch" or args.config == 4:
        run_batch(args)
        return
    if args.workload == "trunc":
        run_trunc(args)
        return

    d, L = args.d, args.primes
    seed = 1003
    # inputs drawn on the device (the distributions of workloads.cpmm_uniform); the CPU baseline
    # reads host copies of the same tensors
    primes, P, A, B = wl.cpmm_uniform_device(seed, d, d, d, args.bits, L)
    p_absmax = 1 << 20
    dev = P.device
    w = None
    if not args.no_cpu_baseline:
        w = types.SimpleNamespace(m=d, k=d, nA=d, nB=d, primes=primes, P=P.cpu().numpy(),
                                  A=A.cpu().numpy().view(np.uint64), B=B.cpu().numpy().view(np.uint64))
    PA = torch.empty((L, d, d), dtype=torch.int64, device=dev)
    PB = torch.empty((L, d, d), dtype=torch.int64, device=dev)
    macs = 2 * L * d * d * d  # mod-q MACs per step

    def step(form):
        return lambda: hlb.cp_mm(P, A, B, primes, p_absmax=p_absmax, form=form, out=(PA, PB))

    def timed(form, names, steps, warmup):
        """Step time of `form` with its kernels bracketed by HIP events on the launch stream."""
        return _profiled(step(form), names, steps, warmup)

    def roofline(kernel, launches, ms, ops_per_step, steps):
        return _roofline(kernel, launches, ms, ops_per_step, steps, d, L, INT8_PEAK_TOPS, "TOP/s", "int8 MAC x 2")

    # Headline: the multimodular INT8 form (Strategy 3; D int8 products per mod-q MAC)
    cplan = hlb.plan(1, d, max(primes), p_absmax, "int8_crt")
    s_crt, kc = timed("int8_crt", ("crt_gemm", "crt_split", "crt_combine"), args.steps,
                      args.warmup)
    c_ops = 2.0 * cplan["p_limbs"] * macs
    out = {
        "metric": METRIC if d == 8192 else METRIC.replace("d=8192", f"d={d}"),
        "value": macs / s_crt,
        "unit": "mod-q MAC/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": s_crt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8", "data": "synthetic",
        "config": {"workload": f"cp_mm d={d}: {d}x{d} plaintext (|P|<=2^20) times {d}x{d} a- and "
                               f"b-parts over {L} RNS primes of {args.bits} bits, INT8-limb form "
                               f"(multimodular: {cplan['p_limbs']} int8 products per mod-q MAC)",
                   "m": d, "k": d, "n": d, "primes": L, "prime_bits": args.bits, "form": "int8_crt",
                   "moduli": cplan["p_limbs"]},
        "roofline": roofline("crt_gemm", kc["crt_gemm"][0], kc["crt_gemm"][1], c_ops, args.steps),
        "kernels_ms": {n: v[1] for n, v in kc.items()},
    }
    # The headline form's output of its last timed step: every other form must reproduce it
    # byte for byte, and the CPU baseline's oracle rows are compared with it.
    ref_PA, ref_PB = PA.clone(), PB.clone()
    identical = {}

    # The digit INT8 form (Strategy 1: 3 x 7 digit products per mod-q MAC)
    if not args.no_digit:
        dplan = hlb.plan(1, d, max(primes), p_absmax, "int8")
        s_dig, kd = timed("int8", ("gemm_i8", "split_p", "split_x"), args.steps, args.warmup)
        d_ops = 2.0 * dplan["p_limbs"] * dplan["x_limbs"] * macs
        out["int8_digit_form"] = {
            "value": macs / s_dig, "unit": "mod-q MAC/s", "ms_per_step": s_dig * 1e3,
            "digits": [dplan["p_limbs"], dplan["x_limbs"]],
            "roofline": roofline("gemm_i8", kd["gemm_i8"][0], kd["gemm_i8"][1], d_ops, args.steps),
            "kernels_ms": {n: v[1] for n, v in kd.items()}}
        identical["int8"] = bool(torch.equal(PA, ref_PA) and torch.equal(PB, ref_PB))

    if not args.no_fp64:
        fp_steps = max(2, args.steps // 3)
        hlb.profile_reset()
        step("fp64")()
        torch.cuda.synchronize()
        hlb.set_option(hlb.OPT_PROFILE, 1)
        s_fp64 = _time_steps(step("fp64"), fp_steps, 0)
        hlb.set_option(hlb.OPT_PROFILE, 0)
        n_f, ms_f = hlb.profile_read("gemm_f64")
        hlb.profile_reset()
        identical["fp64"] = bool(torch.equal(PA, ref_PA) and torch.equal(PB, ref_PB))
        fplan = hlb.plan(1, d, max(primes), p_absmax, "fp64")
        f_ops = 2.0 * fplan["p_limbs"] * fplan["x_limbs"] * macs
        f_tf = f_ops / (ms_f / max(n_f, 1) * 1e-3) / 1e12
        s_dgemm = _dgemm_ms(d, max(3, args.steps // 2)) * 1e-3
        out["fp64_form"] = {"value": macs / s_fp64, "unit": "mod-q MAC/s", "ms_per_step": s_fp64 * 1e3,
                            "limbs": [fplan["p_limbs"], fplan["x_limbs"]], "limb_bits": fplan["limb_bits"],
                            "gemm_tflops": f_tf, "gemm_frac_of_fp64_peak": f_tf / FP64_PEAK_TFLOPS}
        out["fp64_gemm"] = {"ms": s_dgemm * 1e3, "tflops": 2.0 * d ** 3 / s_dgemm / 1e12,
                            "shape": f"{d}x{d}x{d}", "impl": "torch.matmul float64"}
        out["int8_vs_fp64_form_speedup"] = s_fp64 / s_crt
        out["slowdown_vs_fp64_gemm"] = {"int8_form": s_crt / s_dgemm, "fp64_form": s_fp64 / s_dgemm}
        if "int8_digit_form" in out:
            out["slowdown_vs_fp64_gemm"]["int8_digit_form"] = s_dig / s_dgemm

    out["bit_exact"] = {"forms_identical_to_int8_crt": identical}
    ref_host = None
    if w is not None:
        ref_host = (ref_PA.cpu().numpy().view(np.uint64), ref_PB.cpu().numpy().view(np.uint64))
    del ref_PA, ref_PB
    if not args.no_extra_configs:
        del P, A, B, PA, PB
        torch.cuda.empty_cache()
        out["config2_d4096_fp64"] = config2_leg(max(3, args.steps // 2), 2)
        out["config5_d16384_int8"] = config5_leg(max(3, args.steps // 4), 1)
        out["config4_batch64"], _ = batch_leg(args.steps, args.warmup)

    if d == 8192:
        out["paper_figures"] = PAPER_FIGURES
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, ref_host)
        out["bit_exact"]["oracle_rows_equal"] = out["cpu_baseline"]["rows_equal_to_gpu"]

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
