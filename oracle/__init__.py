"""CPU oracle for the CP-MM hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The GPU library never imports it, links it or calls it, and it shares no code with
the GPU library: the two only see the same seeded inputs (from ``workloads``).

Contents
--------
* ``mod_pp_mm``: the definition of Mod-PP-MM_{q; d1,d2,d3} (Section 5): C = P * X mod q,
  computed by the plain C schoolbook in ``oracle.c`` with exact 128-bit accumulation.
* ``cp_mm``: CP-MM as two Mod-PP-MMs per modulus (Algorithm alg:pcmm step 1, Theorem
  th:pcmm-shs), with the plaintext on the left (transpose of the paper's M * U form).
* ``matvec_mod``: matrix-vector product mod q, for Freivalds-style checks at large sizes.
* CKKS helpers written from Section 2.2 (coefficient encoding, Dec) and the row-encryption
  identity A * S + B = Delta * M (mod q) (Eq mat_row_format): ``encode``, ``encrypt``,
  ``decrypt``, ``crt_lift_centered``, ``decode``, ``precision_bits``.
* ``rescale`` (Section 2.2) and ``ccmm_pp_core`` (Algorithm alg:ccmm's plaintext products).
* Strategy 2 of Section 6.1 (truncation), the approximate Mod-PP-MM for the b-part:
  ``mod_pp_mm_drop_i8`` keeps only the digit products of the high shifts (base 256, the
  compromise between Strategies 1 and 2 the paper mentions) and ``mod_pp_mm_trunc_fp64``
  is one floating-point product of the operands rounded to doubles (K = 2^53).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_u64p = ctypes.c_void_p
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64


def build_library(force: bool = False) -> str:
    """Compile oracle.c with gcc (via the Makefile next to it)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "oracle.c"))
    ):
        subprocess.run(["make", "-s", "-B" if force else "-s", "-C", _HERE],
                       check=True, stdout=subprocess.DEVNULL)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build_library()
            lib = ctypes.CDLL(_LIB_PATH)
            lib.oracle_num_threads.restype = ctypes.c_int
            lib.oracle_mod_pp_mm.restype = ctypes.c_int
            lib.oracle_mod_pp_mm.argtypes = [_u64, _i64, _i64, _i64, _u64p, _i64, _u64p, _i64,
                                             _u64p, _i64]
            lib.oracle_mod_pp_mm_rows.restype = ctypes.c_int
            lib.oracle_mod_pp_mm_rows.argtypes = [_u64, _i64, _u64p, _i64, _i64, _u64p, _i64,
                                                  _u64p, _i64, _u64p, _i64]
            lib.oracle_matvec_mod.restype = ctypes.c_int
            lib.oracle_matvec_mod.argtypes = [_u64, _i64, _i64, _u64p, _i64, _u64p, _u64p]
            lib.oracle_residues_of_signed.restype = None
            lib.oracle_residues_of_signed.argtypes = [_u64, _i64, _u64p, _u64p]
            _lib = lib
    return _lib


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().oracle_num_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _as_u64(x) -> np.ndarray:
    a = np.ascontiguousarray(x)
    if a.dtype == np.uint64:
        return a
    if a.dtype.kind in "iu":
        if a.size and int(a.min()) < 0:
            raise ValueError("residue matrix has negative entries")
        return a.astype(np.uint64)
    raise TypeError(f"expected an integer matrix, got {a.dtype}")


def _check(rc: int, what: str):
    if rc == 1:
        raise ValueError(f"{what}: an input entry is not a canonical residue (>= q)")
    if rc != 0:
        raise ValueError(f"{what}: bad arguments")


def mod_pp_mm(q: int, P, X, rows=None) -> np.ndarray:
    """Mod-PP-MM by definition: C[i, j] = sum_l P[i, l] X[l, j] mod q, in [0, q).

    P (m x k) and X (k x n) hold canonical residues.  With ``rows`` given, only those output
    rows are computed (the others are left zero) -- for sampled checks of large products.
    """
    P = _as_u64(P)
    X = _as_u64(X)
    m, k = P.shape
    k2, n = X.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    C = np.zeros((m, n), dtype=np.uint64)
    lib = _load()
    if rows is None:
        rc = lib.oracle_mod_pp_mm(q, m, k, n, _ptr(P), k, _ptr(X), n, _ptr(C), n)
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        if r.size and (r.min() < 0 or r.max() >= m):
            raise ValueError("row index out of range")
        rc = lib.oracle_mod_pp_mm_rows(q, r.size, _ptr(r), k, n, _ptr(P), k, _ptr(X), n,
                                       _ptr(C), n)
    _check(rc, "mod_pp_mm")
    return C


def residues_of_signed(P, q: int) -> np.ndarray:
    """Canonical residues in [0, q) of a signed integer matrix (negative v -> q - |v| mod q)."""
    P = np.ascontiguousarray(np.asarray(P, dtype=np.int64))
    out = np.empty(P.shape, dtype=np.uint64)
    _load().oracle_residues_of_signed(q, P.size, _ptr(P), _ptr(out))
    return out


def cp_mm(P, A, B, primes, rows=None):
    """CP-MM as 2 Mod-PP-MMs per modulus (Algorithm alg:pcmm step 1, Thm th:pcmm-shs).

    P: signed plaintext m x k.  A, B: [L][k][nA], [L][k][nB] residues (or lists of
    per-prime matrices).  Returns (PA, PB) as [L][m][nA], [L][m][nB] uint64 arrays with
    PA[i] = P A[i] mod q_i and PB[i] = P B[i] mod q_i.  No rescaling (boundary reading).
    """
    P = np.asarray(P, dtype=np.int64)
    PA, PB = [], []
    for i, q in enumerate(primes):
        q = int(q)
        Pr = residues_of_signed(P, q)
        PA.append(mod_pp_mm(q, Pr, A[i], rows=rows))
        PB.append(mod_pp_mm(q, Pr, B[i], rows=rows))
    return np.stack(PA), np.stack(PB)


def matvec_mod(q: int, M, v) -> np.ndarray:
    """out = M v mod q for a residue matrix M and residue vector v."""
    M = _as_u64(M)
    v = _as_u64(np.asarray(v).reshape(-1))
    rows, cols = M.shape
    if v.size != cols:
        raise ValueError("vector length differs from matrix columns")
    out = np.empty(rows, dtype=np.uint64)
    _check(_load().oracle_matvec_mod(q, rows, cols, _ptr(M), cols, _ptr(v), _ptr(out)),
           "matvec_mod")
    return out


# ---------------------------------------------------------------------------------------
# CKKS helpers (test-only), written from Section 2.2 and the row-encryption identity.
# ---------------------------------------------------------------------------------------

def round_half_up(x) -> np.ndarray:
    """The paper's rounding: the integer part (floor) of x + 1/2 (Section 2 notation).

    Ties go up (2.5 -> 3, -2.5 -> -2); this is NOT numpy's round-half-to-even.
    """
    return np.floor(np.asarray(x, dtype=np.float64) + 0.5).astype(np.int64)


def encode(M, delta: float) -> np.ndarray:
    """Coefficient encoding of a real matrix: entrywise floor(Delta * m + 1/2)."""
    return round_half_up(np.asarray(M, dtype=np.float64) * float(delta))


def encrypt(A, S, Menc, E, primes):
    """b-part of a fresh encryption: B_i = -A_i S + Menc + E (mod q_i).

    A: [L][k][n] uniform residues, S: n x n small signed secret, Menc: k x n encoded message,
    E: k x n small error.  Then A_i S + B_i = Menc + E (mod q_i), the matrix identity
    A * S + B ~ Delta * M (mod q) in its row form (Eq mat_row_format).
    """
    S = np.asarray(S, dtype=np.int64)
    ME = np.asarray(Menc, dtype=np.int64) + np.asarray(E, dtype=np.int64)
    out = []
    for i, q in enumerate(primes):
        q = int(q)
        AS = mod_pp_mm(q, A[i], residues_of_signed(S, q))
        me = residues_of_signed(ME, q)
        out.append((me + (np.uint64(q) - AS)) % np.uint64(q))
    return np.stack(out)


def decrypt(A, B, S, primes):
    """Dec on a matrix ciphertext: D_i = A_i S + B_i (mod q_i), canonical residues."""
    S = np.asarray(S, dtype=np.int64)
    out = []
    for i, q in enumerate(primes):
        q = int(q)
        AS = mod_pp_mm(q, A[i], residues_of_signed(S, q))
        out.append((AS + np.asarray(B[i], dtype=np.uint64)) % np.uint64(q))
    return np.stack(out)


def crt_lift_centered(D, primes) -> np.ndarray:
    """Chinese remaindering of per-prime residues into the centred range (-Q/2, Q/2].

    D: [L][...] residues.  Returns an object array of Python ints.
    """
    primes = [int(q) for q in primes]
    Q = 1
    for q in primes:
        Q *= q
    acc = np.zeros(np.asarray(D[0]).shape, dtype=object)
    for i, q in enumerate(primes):
        Qi = Q // q
        ci = (Qi * pow(Qi, -1, q)) % Q
        acc = acc + np.asarray(D[i], dtype=np.uint64).astype(object) * ci
    acc = acc % Q
    half = Q // 2
    return np.where(acc > half, acc - Q, acc)


def decode(V, scale: float) -> np.ndarray:
    """Coefficient decoding: the real value p / scale of each integer entry."""
    f = np.vectorize(lambda v: float(v), otypes=[np.float64])
    return f(V) / float(scale)


def precision_bits(M, Mt) -> float:
    """Relative precision log2 ||M||_inf - log2 ||M - Mt||_inf (entrywise max norm).

    Section 6 defines this for the experiment tables; the norm is read as the entrywise
    maximum (the tables quote the worst coefficient).
    """
    M = np.asarray(M, dtype=np.float64)
    err = np.max(np.abs(M - np.asarray(Mt, dtype=np.float64)))
    top = np.max(np.abs(M))
    if err == 0.0:
        return float("inf")
    return float(np.log2(top) - np.log2(err))


def rescale(X, primes):
    """Rescale by the last prime, by definition: for the integer x with residues X[l] (any
    representative modulo the product of the primes), the residues of floor(x / q + 1/2)
    modulo the first L-1 primes, q = primes[L-1] (Section 2.2 Rescale, with the scaling
    factor equal to the dropped prime as Section 5 assumes).  Exact big-integer arithmetic:
    floor(x / q + 1/2) = floor((2x + q) / (2q)).
    """
    primes = [int(p) for p in primes]
    q = primes[-1]
    x = crt_lift_centered(X, primes)          # object array of Python ints
    y = (2 * x + q) // (2 * q)                 # Python floor division of exact integers
    return np.stack([(y % ql).astype(np.uint64) for ql in primes[:-1]])


def ccmm_pp_core(A, B, At, Bt, primes):
    """The four Mod-PP-MMs of the ciphertext-ciphertext product's plaintext core (Algorithm
    alg:ccmm step 2): [A; B] * [At Bt] modulo each prime, returned as (C00, C01, C10, C11)."""
    out = [[], [], [], []]
    for l, q in enumerate(primes):
        q = int(q)
        out[0].append(mod_pp_mm(q, A[l], At[l]))
        out[1].append(mod_pp_mm(q, A[l], Bt[l]))
        out[2].append(mod_pp_mm(q, B[l], At[l]))
        out[3].append(mod_pp_mm(q, B[l], Bt[l]))
    return tuple(np.stack(o) for o in out)


def balanced_digits(v, D: int):
    """The D digits d_0 .. d_{D-1} in [-128, 127] with sum_j d_j 256^j = v (the decomposition
    of Eq decomp with K = 256, digits of either sign).  v: integer array with |v| < 2^62;
    raises ValueError when v needs more than D digits."""
    v = np.asarray(v, dtype=np.int64).copy()
    digits = []
    for _ in range(D):
        d = (v + 128) % 256 - 128          # numpy integer % is a floor modulo
        digits.append(d)
        v = (v - d) // 256                 # exact: v - d is a multiple of 256
    if np.any(v != 0):
        raise ValueError(f"value needs more than {D} balanced base-256 digits")
    return digits


def mod_pp_mm_drop_i8(q: int, P, X, drop: int, dp: int, dx: int) -> np.ndarray:
    """Truncated Mod-PP-MM in base 256: with P = sum_i P_i 256^i (dp signed digits of the
    signed plaintext) and X = sum_j X_j 256^j (dx digits of the residues), the integer
    sum over i + j >= drop of (P_i X_j) 256^(i+j), reduced mod q -- Strategy 2 of Section
    6.1 keeping only the terms of the decomposition above shift `drop`."""
    q = int(q)
    Pd = balanced_digits(P, dp)
    Xd = balanced_digits(np.asarray(X, dtype=np.uint64).astype(np.int64), dx)
    total = np.zeros((np.shape(P)[0], np.shape(X)[1]), dtype=object)
    for i in range(dp):
        for j in range(dx):
            if i + j >= drop:
                # each entry is a sum of k products of two digits: |.| <= k 2^14, exact in int64
                total = total + (Pd[i] @ Xd[j]).astype(object) * (256 ** (i + j))
    return np.array([[int(t) % q for t in row] for row in total], dtype=np.uint64)


def centred(X, q: int) -> np.ndarray:
    """Centred representatives in (-q/2, q/2] of residues X in [0, q)."""
    X = np.asarray(X, dtype=np.uint64).astype(np.int64)
    return np.where(2 * X > int(q), X - int(q), X)


def mod_pp_mm_trunc_fp64(q: int, P, X) -> np.ndarray:
    """Strategy 2 of Section 6.1 with K = 2^53: round both operands to doubles (the signed
    plaintext P, the residues X in their centred representatives), multiply them with one
    floating-point matrix product, and return the canonical residue mod q of the result.
    The product's entries are integer-valued doubles (every rounding of an integer of
    magnitude >= 2^53 is again an integer), so the residue is well defined."""
    q = int(q)
    Pt = np.asarray(P, dtype=np.int64).astype(np.float64)
    Xt = centred(X, q).astype(np.float64)
    Y = Pt @ Xt
    if not np.all(np.isfinite(Y)) or not np.all(Y == np.floor(Y)):
        raise ValueError("floating-point product is not integer-valued")
    return np.array([[int(y) % q for y in row] for row in Y.tolist()], dtype=np.uint64)
