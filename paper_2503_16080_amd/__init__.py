"""Python binding of libhlb: bit-exact CKKS ciphertext-plaintext matrix products on MI355X.

A thin ctypes layer over the C ABI in ``include/hlb.h``: argument marshalling only, every
step of the computation runs in the library's HIP kernels.  PyTorch supplies device memory
(residues live in int64 or uint64 CUDA tensors, bit-identical since residues < 2^52) and the
stream (``torch.cuda.current_stream()``).

The binding exposes functions with the C names (``hlb_mod_pp_mm``, ``hlb_cp_mm``, ...) taking
tensors, plus short aliases (``mod_pp_mm``, ``cp_mm``, ...).  There is no fallback: if
libhlb.so is missing or fails to load, every call raises ``HlbError``.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Sequence

import torch

__all__ = [
    "HlbError", "FORM_AUTO", "FORM_FP64", "FORM_INT8", "library_path", "load",
    "hlb_mod_pp_mm", "hlb_cp_mm", "hlb_cp_mm_noalloc", "hlb_cp_mm_batch", "hlb_validate_residues",
    "hlb_plaintext_absmax", "hlb_plan", "hlb_set_option", "hlb_profile_read",
    "hlb_profile_reset", "hlb_release", "hlb_status_str", "hlb_test_encode",
    "hlb_test_encrypt", "hlb_test_decrypt", "hlb_tune_set", "hlb_tune_load", "hlb_tune_class",
    "hlb_tune_set_crt", "hlb_tune_class_crt",
    "hlb_ccmm_pp_core", "hlb_rescale", "ccmm_pp_core", "rescale",
    "mod_pp_mm", "cp_mm", "cp_mm_noalloc", "cp_mm_batch", "validate_residues", "plaintext_absmax", "plan",
    "set_option", "profile_read", "profile_reset", "release",
]

FORM_AUTO, FORM_FP64, FORM_INT8, FORM_INT8_CRT = 0, 1, 2, 3
_FORMS = {"auto": FORM_AUTO, "fp64": FORM_FP64, "int8": FORM_INT8, "int8_crt": FORM_INT8_CRT}
OPT_FORCE_KCHUNK, OPT_PROFILE, OPT_BATCH_GRAPH, OPT_FORCE_CLASS, OPT_F64_PLANES, OPT_CRT_WIDE = 1, 2, 3, 4, 5, 6
OPT_WS_CAP = 7
OPT_VALIDATE = 8
NOALLOC_SCRATCH_BYTES = 256 << 20   # HLB_NOALLOC_SCRATCH_BYTES

_HERE = os.path.dirname(os.path.abspath(__file__))
# HLB_LIBRARY selects another build of the same library (the host-sanitizer build)
_LIB_PATH = os.environ.get("HLB_LIBRARY") or os.path.join(_HERE, "libhlb.so")
_lib = None
_lock = threading.Lock()


class HlbError(RuntimeError):
    """A libhlb call failed (status code and message), or the library is unavailable."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"hlb status {status}: {msg}")
        self.status = status


def library_path() -> str:
    return _LIB_PATH


class PlanDesc(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("p_limbs", ctypes.c_int), ("x_limbs", ctypes.c_int),
                ("shifts", ctypes.c_int), ("limb_bits", ctypes.c_int), ("max_pairs", ctypes.c_int),
                ("k_chunk", ctypes.c_int64), ("acc_bound_log2", ctypes.c_double)]


class TruncDesc(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("truncated", ctypes.c_int), ("dropped_shifts", ctypes.c_int),
                ("products", ctypes.c_int), ("err_bound_log2", ctypes.c_double)]


class CpmmProblem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int64), ("nA", ctypes.c_int64),
                ("nB", ctypes.c_int64), ("P", ctypes.c_void_p), ("ldp", ctypes.c_int64),
                ("p_absmax", ctypes.c_int64), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("PA", ctypes.c_void_p), ("PB", ctypes.c_void_p)]


def load():
    """Loads libhlb.so (once).  Raises HlbError when it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise HlbError(-1, f"{_LIB_PATH} is not built; run python -m paper_2503_16080_amd._build")
        try:
            lib = ctypes.CDLL(_LIB_PATH)
        except OSError as e:
            raise HlbError(-1, f"cannot load {_LIB_PATH}: {e}") from e
        i64, u64, vp, ci = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        sig = {
            "hlb_status_str": (ctypes.c_char_p, [ci]),
            "hlb_mod_pp_mm": (ci, [u64, i64, i64, i64, vp, i64, vp, i64, vp, i64, ci, vp]),
            "hlb_cp_mm": (ci, [i64, i64, i64, i64, vp, i64, i64, vp, vp, vp, ci, vp, vp, ci, vp]),
            "hlb_cp_mm_noalloc": (ci, [i64, i64, i64, i64, vp, i64, i64, vp, vp, vp, ci, vp, vp, ci, vp]),
            "hlb_cp_mm_trunc_b": (ci, [i64, i64, i64, i64, vp, i64, i64, vp, vp, vp, ci, vp, vp,
                                       ctypes.c_double, ci, vp]),
            "hlb_plan_trunc_b": (ci, [i64, u64, u64, i64, ctypes.c_double, ci, vp]),
            "hlb_cp_mm_batch": (ci, [vp, ci, vp, ci, ci, vp]),
            "hlb_validate_residues": (ci, [vp, i64, i64, i64, u64, vp, vp]),
            "hlb_plaintext_absmax": (ci, [vp, i64, i64, i64, vp, vp]),
            "hlb_plan": (ci, [ci, i64, u64, i64, ci, vp]),
            "hlb_set_option": (ci, [ci, i64]),
            "hlb_profile_read": (ci, [ctypes.c_char_p, vp, vp]),
            "hlb_profile_reset": (ci, []),
            "hlb_release": (ci, []),
            "hlb_test_encode": (ci, [vp, i64, ctypes.c_double, vp, vp]),
            "hlb_test_encrypt": (ci, [i64, i64, vp, vp, vp, vp, ci, vp, vp]),
            "hlb_test_decrypt": (ci, [i64, i64, vp, vp, vp, vp, ci, vp, vp]),
            "hlb_ccmm_pp_core": (ci, [i64, i64, i64, vp, vp, vp, vp, vp, ci, vp, vp, vp, vp, ci, vp]),
            "hlb_rescale": (ci, [i64, vp, vp, ci, vp, vp]),
            "hlb_tune_set": (ci, [ci, ci, ci, ci, ci]),
            "hlb_tune_load": (ci, [ctypes.c_char_p]),
            "hlb_tune_class": (ci, [ci, i64, i64, i64]),
            "hlb_tune_set_crt": (ci, [ci, ci, ci, ci, ci]),
            "hlb_tune_class_crt": (ci, [ci, i64, i64, i64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def hlb_status_str(status: int) -> str:
    return load().hlb_status_str(int(status)).decode()


def _check(status: int, what: str):
    if status != 0:
        raise HlbError(status, f"{what}: {hlb_status_str(status)}")


def _form(form) -> int:
    if isinstance(form, str):
        return _FORMS[form.lower()]
    return int(form)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _int64(t, name: str) -> torch.Tensor:
    """A 64-bit integer tensor (int64 or uint64; residues < 2^52 are bit-identical in both)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"{name} must be int64 or uint64, got {t.dtype}")
    return t


def _shape(t, name: str, shape) -> torch.Tensor:
    """Checks dtype and exact shape (ValueError on a shape mismatch) -- no device access."""
    _int64(t, name)
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _on_device(ref: torch.Tensor, *named) -> None:
    """Every tensor must live on the same CUDA device as `ref` (checked after the shapes, so
    that shape errors are reported before anything touches a device)."""
    if not ref.is_cuda:
        raise TypeError("operands must be CUDA tensors")
    for t, name in named:
        if not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.device != ref.device:
            raise ValueError(f"{name} is on {t.device}, the operands on {ref.device}")


def _dev64(t: torch.Tensor, name: str) -> torch.Tensor:
    _int64(t, name)
    if not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    return t


def _row_stride(t: torch.Tensor, name: str) -> int:
    if t.dim() == 2 and t.numel() == 0:
        return t.shape[1]  # no element is addressed; any stride >= the row length is valid
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major view (unit column stride)")
    return max(t.stride(0), t.shape[1])


# ------------------------------------------------------------------------------------------
# Product entry points
# ------------------------------------------------------------------------------------------

def hlb_mod_pp_mm(q: int, P: torch.Tensor, X: torch.Tensor, form="auto", out=None, stream=None):
    """C = P X mod q (Mod-PP-MM).  P: m x k residues, X: k x n residues; returns m x n."""
    _int64(P, "P")
    _int64(X, "X")
    if P.dim() != 2 or X.dim() != 2:
        raise ValueError("P and X must be 2-D")
    m, k = P.shape
    k2, n = X.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if out is not None:
        _shape(out, "out", (m, n))
    _on_device(P, (X, "X"), *(((out, "out"),) if out is not None else ()))
    C = out if out is not None else torch.empty((m, n), dtype=torch.int64, device=P.device)
    _check(load().hlb_mod_pp_mm(int(q), m, k, n, P.data_ptr(), _row_stride(P, "P"), X.data_ptr(),
                                _row_stride(X, "X"), C.data_ptr(), _row_stride(C, "out"),
                                _form(form), _stream(stream)), "mod_pp_mm")
    return C


def _cp_mm_operands(P, A, B, primes, out):
    _int64(P, "P")
    _int64(A, "A")
    _int64(B, "B")
    L = len(primes)
    if P.dim() != 2:
        raise ValueError("P must be 2-D (m x k)")
    m, k = P.shape
    if A.dim() != 3 or B.dim() != 3 or A.shape[0] != L or B.shape[0] != L or A.shape[1] != k \
            or B.shape[1] != k:
        raise ValueError("A and B must be [L, k, n] with L = len(primes)")
    nA, nB = A.shape[2], B.shape[2]
    if out is not None:
        PA, PB = out
        _shape(PA, "PA", (L, m, nA))
        _shape(PB, "PB", (L, m, nB))
    _on_device(P, (A, "A"), (B, "B"), *(((PA, "PA"), (PB, "PB")) if out is not None else ()))
    if not (A.is_contiguous() and B.is_contiguous()):
        raise ValueError("A and B must be contiguous")
    if out is None:
        PA = torch.empty((L, m, nA), dtype=torch.int64, device=P.device)
        PB = torch.empty((L, m, nB), dtype=torch.int64, device=P.device)
    elif not (PA.is_contiguous() and PB.is_contiguous()):
        raise ValueError("outputs must be contiguous")
    qs = (ctypes.c_uint64 * max(L, 1))(*[int(q) for q in primes])
    return (m, k, nA, nB, P.data_ptr(), _row_stride(P, "P")), (A.data_ptr(), B.data_ptr(), qs, L,
                                                              PA.data_ptr(), PB.data_ptr()), PA, PB


def hlb_cp_mm(P: torch.Tensor, A: torch.Tensor, B: torch.Tensor, primes: Sequence[int],
              p_absmax: int = 0, form="int8", out=None, stream=None):
    """(P A_l mod q_l, P B_l mod q_l) for every prime (CP-MM over an RNS basis).

    P: m x k signed int64; A: [L, k, nA], B: [L, k, nB] residues (contiguous).  Returns
    (PA, PB) of shapes [L, m, nA], [L, m, nB].  p_absmax = 0 measures max |P| on the device.
    """
    head, tail, PA, PB = _cp_mm_operands(P, A, B, primes, out)
    _check(load().hlb_cp_mm(*head, int(p_absmax), *tail, _form(form), _stream(stream)), "cp_mm")
    return PA, PB


def hlb_cp_mm_noalloc(P: torch.Tensor, A: torch.Tensor, B: torch.Tensor, primes: Sequence[int],
                      p_absmax: int, form="int8", out=None, stream=None):
    """hlb_cp_mm with every workspace buffer in the library's static scratch array (no device
    allocation in the library; HLB_NOALLOC_SCRATCH_BYTES per device).  p_absmax must be >= 1.
    Pass `out` to keep the call itself allocation-free (otherwise the outputs are allocated
    here, by torch, before the call)."""
    head, tail, PA, PB = _cp_mm_operands(P, A, B, primes, out)
    _check(load().hlb_cp_mm_noalloc(*head, int(p_absmax), *tail, _form(form), _stream(stream)), "cp_mm_noalloc")
    return PA, PB


def hlb_cp_mm_trunc_b(P: torch.Tensor, A: torch.Tensor, B: torch.Tensor, primes: Sequence[int],
                      b_err_log2: float, p_absmax: int = 0, form="int8", out=None, stream=None):
    """CP-MM with the a-part exact and the b-part within 2^b_err_log2 of the exact residue
    (Strategy 2 of Section 6.1); arguments and results as for hlb_cp_mm."""
    head, tail, PA, PB = _cp_mm_operands(P, A, B, primes, out)
    _check(load().hlb_cp_mm_trunc_b(*head, int(p_absmax), *tail, float(b_err_log2), _form(form),
                                    _stream(stream)), "cp_mm_trunc_b")
    return PA, PB


def hlb_plan_trunc_b(k: int, q_min: int, q_max: int, p_absmax: int, b_err_log2: float,
                     form="int8") -> dict:
    """The b-part plan hlb_cp_mm_trunc_b would take (host only)."""
    d = TruncDesc()
    _check(load().hlb_plan_trunc_b(int(k), int(q_min), int(q_max), int(p_absmax),
                                   float(b_err_log2), _form(form), ctypes.byref(d)), "plan_trunc_b")
    return {f: getattr(d, f) for f, _ in TruncDesc._fields_}


def hlb_cp_mm_batch(problems, primes: Sequence[int], form="int8", stream=None):
    """A batch of CP-MMs sharing the primes.

    problems: list of dicts with keys P, A, B, and optionally p_absmax, PA, PB (outputs are
    allocated when absent).  Returns the list of (PA, PB).
    """
    L = len(primes)
    # shapes of every problem first, then devices: a bad member fails before any allocation
    ref = None
    for i, pr in enumerate(problems):
        P, A, B = _int64(pr["P"], f"P[{i}]"), _int64(pr["A"], f"A[{i}]"), _int64(pr["B"], f"B[{i}]")
        if P.dim() != 2:
            raise ValueError(f"P of problem {i} must be 2-D (m x k)")
        m, k = P.shape
        if A.dim() != 3 or B.dim() != 3 or tuple(A.shape[:2]) != (L, k) or tuple(B.shape[:2]) != (L, k):
            raise ValueError(f"A and B of problem {i} must be [L, k, n] with L = len(primes), k = {k}")
        if pr.get("PA") is not None:
            _shape(pr["PA"], f"PA[{i}]", (L, m, A.shape[2]))
        if pr.get("PB") is not None:
            _shape(pr["PB"], f"PB[{i}]", (L, m, B.shape[2]))
        ref = P if ref is None else ref
    for i, pr in enumerate(problems):
        _on_device(ref, *((pr[key], f"{key}[{i}]") for key in ("P", "A", "B", "PA", "PB")
                          if pr.get(key) is not None))
    arr = (CpmmProblem * max(len(problems), 1))()
    outs = []
    for i, pr in enumerate(problems):
        P, A, B = pr["P"], pr["A"], pr["B"]
        m, k = P.shape
        nA, nB = A.shape[2], B.shape[2]
        PA = pr.get("PA")
        PB = pr.get("PB")
        if PA is None:
            PA = torch.empty((L, m, nA), dtype=torch.int64, device=P.device)
        if PB is None:
            PB = torch.empty((L, m, nB), dtype=torch.int64, device=P.device)
        for t, nm in ((A, "A"), (B, "B"), (PA, "PA"), (PB, "PB")):
            if not t.is_contiguous():
                raise ValueError(f"{nm} of problem {i} must be contiguous")
        arr[i] = CpmmProblem(m, k, nA, nB, P.data_ptr(), _row_stride(P, "P"),
                             int(pr.get("p_absmax", 0)), A.data_ptr(), B.data_ptr(),
                             PA.data_ptr(), PB.data_ptr())
        outs.append((PA, PB))
    qs = (ctypes.c_uint64 * max(L, 1))(*[int(q) for q in primes])
    _check(load().hlb_cp_mm_batch(ctypes.cast(arr, ctypes.c_void_p), len(problems), qs, L,
                                  _form(form), _stream(stream)), "cp_mm_batch")
    return outs


def hlb_ccmm_pp_core(A, B, At, Bt, primes: Sequence[int], form="auto", stream=None):
    """[A; B] * [At Bt] modulo each prime (CC-MM plaintext core): returns (C00, C01, C10, C11),
    each [L, m, n].  A, B: [L, m, k]; At, Bt: [L, k, n]; all contiguous residue tensors."""
    for t, nm in ((A, "A"), (B, "B"), (At, "At"), (Bt, "Bt")):
        _int64(t, nm)
        if t.dim() != 3:
            raise ValueError(f"{nm} must be a contiguous [L, rows, cols] tensor")
    L = len(primes)
    _, m, k = A.shape
    n = At.shape[2]
    if B.shape != A.shape or Bt.shape != At.shape or At.shape[1] != k or A.shape[0] != L or At.shape[0] != L:
        raise ValueError("shapes must be A, B: [L, m, k] and At, Bt: [L, k, n]")
    _on_device(A, (B, "B"), (At, "At"), (Bt, "Bt"))
    for t, nm in ((A, "A"), (B, "B"), (At, "At"), (Bt, "Bt")):
        if not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous [L, rows, cols] tensor")
    outs = [torch.empty((L, m, n), dtype=torch.int64, device=A.device) for _ in range(4)]
    qs = (ctypes.c_uint64 * max(L, 1))(*[int(q) for q in primes])
    _check(load().hlb_ccmm_pp_core(m, k, n, A.data_ptr(), B.data_ptr(), At.data_ptr(), Bt.data_ptr(), qs, L,
                                   *[o.data_ptr() for o in outs], _form(form), _stream(stream)), "ccmm_pp_core")
    return tuple(outs)


def hlb_rescale(X, primes: Sequence[int], stream=None):
    """Rescale by the last prime: X is [L, ...] residues of integers x; returns [L-1, ...]
    residues of floor(x / q_{L-1} + 1/2)."""
    _dev64(X, "X")
    if not X.is_contiguous() or X.shape[0] != len(primes):
        raise ValueError("X must be contiguous with leading dimension L = len(primes)")
    L = len(primes)
    count = X[0].numel() if L else 0
    Y = torch.empty((max(L - 1, 0),) + tuple(X.shape[1:]), dtype=torch.int64, device=X.device)
    qs = (ctypes.c_uint64 * max(L, 1))(*[int(q) for q in primes])
    _check(load().hlb_rescale(count, X.data_ptr(), qs, L, Y.data_ptr(), _stream(stream)), "rescale")
    return Y


def hlb_validate_residues(X: torch.Tensor, q: int, stream=None) -> int:
    """Synchronous: returns -1 when every entry is < q, else the first offending index."""
    _dev64(X, "X")
    rows, cols = X.shape
    bad = ctypes.c_int64(-1)
    st = load().hlb_validate_residues(X.data_ptr(), rows, cols, _row_stride(X, "X"), int(q),
                                      ctypes.byref(bad), _stream(stream))
    if st not in (0, 2):
        _check(st, "validate_residues")
    return int(bad.value)


def hlb_plaintext_absmax(P: torch.Tensor, stream=None) -> int:
    _dev64(P, "P")
    m, k = P.shape
    v = ctypes.c_int64(0)
    _check(load().hlb_plaintext_absmax(P.data_ptr(), m, k, _row_stride(P, "P"), ctypes.byref(v),
                                       _stream(stream)), "plaintext_absmax")
    return int(v.value)


def hlb_plan(kind: int, k: int, q_max: int, p_absmax: int = 1, form="auto") -> dict:
    """The limb plan the library would use (host only; kind 0 = Mod-PP-MM, 1 = CP-MM)."""
    d = PlanDesc()
    _check(load().hlb_plan(int(kind), int(k), int(q_max), int(p_absmax), _form(form),
                           ctypes.byref(d)), "plan")
    return {f: getattr(d, f) for f, _ in PlanDesc._fields_}


def hlb_set_option(option: int, value: int):
    _check(load().hlb_set_option(int(option), int(value)), "set_option")


def hlb_profile_read(name: str):
    """(launches, total_ms) of kernel class `name` recorded while profiling was on."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(load().hlb_profile_read(name.encode(), ctypes.byref(n), ctypes.byref(ms)), "profile_read")
    return int(n.value), float(ms.value)


def hlb_profile_reset():
    _check(load().hlb_profile_reset(), "profile_reset")


def hlb_release():
    _check(load().hlb_release(), "release")


def hlb_tune_set(x_digits: int, log2m: int, log2n: int, log2k: int, cls: int):
    _check(load().hlb_tune_set(int(x_digits), int(log2m), int(log2n), int(log2k), int(cls)), "tune_set")


def hlb_tune_load(path: str):
    _check(load().hlb_tune_load(path.encode()), "tune_load")


def hlb_tune_class(x_digits: int, m: int, n: int, k: int) -> int:
    """INT8 tile class the planner picks for an m x n (one output matrix) x k problem."""
    return int(load().hlb_tune_class(int(x_digits), int(m), int(n), int(k)))


def hlb_tune_set_crt(moduli: int, log2m: int, log2n: int, log2k: int, cls: int):
    _check(load().hlb_tune_set_crt(int(moduli), int(log2m), int(log2n), int(log2k), int(cls)), "tune_set_crt")


def hlb_tune_class_crt(moduli: int, m: int, n: int, k: int) -> int:
    """Multimodular tile class (0: 256 x 128, 1: 256 x 256, 2: 256 x 384 outputs) the planner
    picks for an m x n (one output matrix) x k problem over `moduli` moduli."""
    return int(load().hlb_tune_class_crt(int(moduli), int(m), int(n), int(k)))


# ------------------------------------------------------------------------------------------
# Test-only helpers
# ------------------------------------------------------------------------------------------

def hlb_test_encode(M: torch.Tensor, delta: float, stream=None) -> torch.Tensor:
    if M.dtype != torch.float64 or not M.is_cuda or not M.is_contiguous():
        raise TypeError("M must be a contiguous float64 CUDA tensor")
    out = torch.empty(M.shape, dtype=torch.int64, device=M.device)
    _check(load().hlb_test_encode(M.data_ptr(), M.numel(), float(delta), out.data_ptr(),
                                  _stream(stream)), "test_encode")
    return out


def hlb_test_encrypt(A: torch.Tensor, S: torch.Tensor, Menc: torch.Tensor, primes, stream=None):
    _int64(A, "A")
    if A.dim() != 3 or A.shape[0] != len(primes):
        raise ValueError("A must be [L, k, n] with L = len(primes)")
    L, k, n = A.shape
    _shape(S, "S", (n, n))
    _shape(Menc, "Menc", (k, n))
    _on_device(A, (S, "S"), (Menc, "Menc"))
    for t, nm in ((A, "A"), (S, "S"), (Menc, "Menc")):
        if not t.is_contiguous():
            raise ValueError(f"{nm} must be contiguous")
    B = torch.empty_like(A)
    qs = (ctypes.c_uint64 * max(L, 1))(*[int(q) for q in primes])
    _check(load().hlb_test_encrypt(k, n, A.data_ptr(), S.data_ptr(), Menc.data_ptr(), qs, L,
                                   B.data_ptr(), _stream(stream)), "test_encrypt")
    return B


def hlb_test_decrypt(A: torch.Tensor, B: torch.Tensor, S: torch.Tensor, primes, stream=None):
    _int64(A, "A")
    if A.dim() != 3 or A.shape[0] != len(primes):
        raise ValueError("A must be [L, rows, n] with L = len(primes)")
    L, rows, n = A.shape
    _shape(B, "B", tuple(A.shape))
    _shape(S, "S", (n, n))
    _on_device(A, (B, "B"), (S, "S"))
    for t, nm in ((A, "A"), (B, "B"), (S, "S")):
        if not t.is_contiguous():
            raise ValueError(f"{nm} must be contiguous")
    D = torch.empty_like(A)
    qs = (ctypes.c_uint64 * max(L, 1))(*[int(q) for q in primes])
    _check(load().hlb_test_decrypt(rows, n, A.data_ptr(), B.data_ptr(), S.data_ptr(), qs, L,
                                   D.data_ptr(), _stream(stream)), "test_decrypt")
    return D


# short aliases
ccmm_pp_core = hlb_ccmm_pp_core
rescale = hlb_rescale
mod_pp_mm = hlb_mod_pp_mm
cp_mm = hlb_cp_mm
cp_mm_trunc_b = hlb_cp_mm_trunc_b
cp_mm_noalloc = hlb_cp_mm_noalloc
plan_trunc_b = hlb_plan_trunc_b
cp_mm_batch = hlb_cp_mm_batch
validate_residues = hlb_validate_residues
plaintext_absmax = hlb_plaintext_absmax
plan = hlb_plan
set_option = hlb_set_option
profile_read = hlb_profile_read
profile_reset = hlb_profile_reset
release = hlb_release
