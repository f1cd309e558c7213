"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the CPU oracle.

This module only draws random numbers and picks moduli; it holds none of the modular
matrix-product arithmetic.  Every generator takes an explicit seed (numpy PCG64), so the GPU
side and the oracle side see bit-identical inputs.

The distributions follow the paper's matrix experiments (Section 6.3: entries i.i.d.
uniform in [-1, 1], plaintext scale about 2^20) and the standard CKKS ingredients (Section
2.2): uniform a-parts modulo each prime, a ternary secret, a rounded Gaussian error.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Deterministic Miller-Rabin: these 12 prime bases decide primality exactly for every
# n < 3.3e24 (Sorenson and Webster, 2015), which covers all moduli used here (< 2^62).
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(bits: int, count: int, skip: int = 0, two_adicity: int = 17) -> list[int]:
    """The `count` largest primes q < 2^bits with q = 1 (mod 2^two_adicity), after skipping
    the first `skip` of them (so a seed can select a different set)."""
    if bits <= two_adicity + 1:
        raise ValueError("bits too small for the requested 2-adicity")
    step = 1 << two_adicity
    q = ((1 << bits) - 1) // step * step + 1
    if q >= (1 << bits):
        q -= step
    out: list[int] = []
    seen = 0
    while len(out) < count:
        if q < (1 << (bits - 1)):
            raise ValueError("ran out of primes in range")
        if is_prime(q):
            if seen >= skip:
                out.append(q)
            seen += 1
        q -= step
    return out


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_residues(g: np.random.Generator, shape, q: int) -> np.ndarray:
    """Entries i.i.d. uniform in [0, q), as uint64."""
    return g.integers(0, q, size=shape, dtype=np.uint64)


def uniform_real(g: np.random.Generator, shape) -> np.ndarray:
    """Entries i.i.d. uniform in [-1, 1] (float64)."""
    return g.uniform(-1.0, 1.0, size=shape)


def plaintext_matrix(g: np.random.Generator, m: int, k: int, scale_bits: int = 20) -> np.ndarray:
    """Fixed-point plaintext P = floor(2^scale_bits * U + 1/2), U uniform in [-1, 1].

    |P| <= 2^scale_bits.  Returned as int64."""
    U = uniform_real(g, (m, k))
    return np.floor(U * float(1 << scale_bits) + 0.5).astype(np.int64)


def ternary(g: np.random.Generator, shape) -> np.ndarray:
    """Uniform ternary entries in {-1, 0, 1} (int64)."""
    return g.integers(-1, 2, size=shape, dtype=np.int64)


def rounded_gaussian(g: np.random.Generator, shape, sigma: float = 3.2) -> np.ndarray:
    """floor(N(0, sigma^2) + 1/2), no tail cut (int64)."""
    return np.floor(g.normal(0.0, sigma, size=shape) + 0.5).astype(np.int64)


@dataclass
class CpmmWorkload:
    """One CP-MM problem: plaintext P (m x k) and a ciphertext (A, B) over L primes."""
    m: int
    k: int
    nA: int
    nB: int
    primes: list[int]
    P: np.ndarray            # int64 m x k, |P| <= p_absmax
    A: np.ndarray            # uint64 [L][k][nA]
    B: np.ndarray            # uint64 [L][k][nB]
    p_absmax: int
    extra: dict = field(default_factory=dict)


def cpmm_uniform(seed: int, m: int, k: int, n: int, bits: int, L: int,
                 scale_bits: int = 20, nB: int | None = None) -> CpmmWorkload:
    """CP-MM inputs with the a- and b-parts drawn uniform modulo each prime.

    A b-part of an RLWE-type ciphertext is computationally indistinguishable from uniform,
    and the product kernels are data-independent, so this is the timing workload; the
    end-to-end test builds a real encryption instead (see the oracle's encrypt helper).
    """
    g = rng(seed)
    primes = ntt_primes(bits, L, skip=seed % 8)
    nB = n if nB is None else nB
    P = plaintext_matrix(g, m, k, scale_bits)
    A = np.stack([uniform_residues(g, (k, n), q) for q in primes]) if L else \
        np.zeros((0, k, n), np.uint64)
    B = np.stack([uniform_residues(g, (k, nB), q) for q in primes]) if L else \
        np.zeros((0, k, nB), np.uint64)
    return CpmmWorkload(m, k, n, nB, primes, P, A, B, 1 << scale_bits)


@dataclass
class CkksInputs:
    """Raw draws for an end-to-end CKKS check: message M, secret S, error E, a-parts A."""
    M: np.ndarray     # float64 k x n, uniform [-1, 1]
    S: np.ndarray     # int64 n x n ternary
    E: np.ndarray     # int64 k x n rounded Gaussian
    A: np.ndarray     # uint64 [L][k][n] uniform residues
    U: np.ndarray     # float64 m x k, uniform [-1, 1] (plaintext before scaling)
    primes: list[int]
    delta_bits: int
    p_scale_bits: int


def ckks_draws(seed: int, m: int, k: int, n: int, bits: int, L: int,
               delta_bits: int = 40, p_scale_bits: int = 20, sigma: float = 3.2) -> CkksInputs:
    g = rng(seed)
    primes = ntt_primes(bits, L, skip=seed % 8)
    M = uniform_real(g, (k, n))
    S = ternary(g, (n, n))
    E = rounded_gaussian(g, (k, n), sigma)
    A = np.stack([uniform_residues(g, (k, n), q) for q in primes])
    U = uniform_real(g, (m, k))
    return CkksInputs(M, S, E, A, U, primes, delta_bits, p_scale_bits)


def batch_shapes(seed: int, count: int = 64, d_lo: int = 128, d_hi: int = 4096,
                 m_lo: int = 64, m_hi: int = 4096) -> list[tuple[int, int]]:
    """(m, d) pairs with d and m drawn log-uniformly, rounded to integers."""
    g = rng(seed)
    out = []
    for _ in range(count):
        d = int(round(math.exp(g.uniform(math.log(d_lo), math.log(d_hi)))))
        m = int(round(math.exp(g.uniform(math.log(m_lo), math.log(m_hi)))))
        out.append((m, d))
    return out


# The five benchmark/test configurations of the CP-MM hot path.
CONFIGS = {
    1: dict(kind="mod_pp_mm", m=256, k=256, n=256, bits=50, L=1, form="fp64", seed=1001),
    2: dict(kind="cp_mm", d=4096, bits=50, L=3, form="fp64", seed=1002),
    3: dict(kind="cp_mm", d=8192, bits=50, L=3, form="int8", seed=1003),
    4: dict(kind="cp_mm_batch", count=64, bits=45, L=4, form="int8", seed=1004),
    5: dict(kind="cp_mm", d=16384, bits=50, L=2, form="int8", seed=1005),
}


# ---------------------------------------------------------------------------------------
# Device-side generators for the large configurations: the same distributions, drawn with a
# seeded torch generator on the GPU (a d = 16384 ciphertext is 10 GiB of residues, too slow to
# draw on the host).  Both the library and the oracle see these exact tensors: the checks copy
# them to the host.
# ---------------------------------------------------------------------------------------

def device_generator(seed: int, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def plaintext_matrix_device(g, m: int, k: int, scale_bits: int = 20, device="cuda"):
    """P = floor(2^scale_bits * U + 1/2) with U uniform in [-1, 1], int64 on the device."""
    import torch
    U = torch.rand((m, k), dtype=torch.float64, device=device, generator=g) * 2.0 - 1.0
    return torch.floor(U * float(1 << scale_bits) + 0.5).to(torch.int64)


def uniform_residues_device(g, shape, q: int, device="cuda"):
    """Entries uniform in [0, q), int64 on the device (bit-identical to uint64 residues)."""
    import torch
    return torch.randint(0, int(q), tuple(shape), dtype=torch.int64, device=device, generator=g)


def cpmm_uniform_device(seed: int, m: int, k: int, n: int, bits: int, L: int, scale_bits: int = 20,
                        device="cuda"):
    """(primes, P, A, B) of a CP-MM drawn on the device: the distributions of cpmm_uniform."""
    import torch
    g = device_generator(seed, device)
    primes = ntt_primes(bits, L, skip=seed % 8)
    P = plaintext_matrix_device(g, m, k, scale_bits, device)
    A = torch.stack([uniform_residues_device(g, (k, n), q, device) for q in primes])
    B = torch.stack([uniform_residues_device(g, (k, n), q, device) for q in primes])
    return primes, P, A, B


def batch_problems_device(seed: int = 1004, count: int = 64, bits: int = 45, L: int = 4,
                          scale_bits: int = 20, device="cuda"):
    """The batch workload: `count` CP-MMs with (m, d) from batch_shapes(seed), n = d, over the
    L primes of `bits` bits; returns (primes, shapes, problems) with problems as dicts of
    device tensors P (m x d), A and B ([L][d][d])."""
    g = device_generator(seed, device)
    primes = ntt_primes(bits, L, skip=seed % 8)
    shapes = batch_shapes(seed, count)
    probs = []
    import torch
    for (m, d) in shapes:
        P = plaintext_matrix_device(g, m, d, scale_bits, device)
        A = torch.stack([uniform_residues_device(g, (d, d), q, device) for q in primes])
        B = torch.stack([uniform_residues_device(g, (d, d), q, device) for q in primes])
        probs.append(dict(P=P, A=A, B=B, p_absmax=1 << scale_bits))
    return primes, shapes, probs
