"""The recombination of the multimodular form, emulated on the CPU in the integer arithmetic the
kernel performs: byte dot products of the coefficients y_i with the bytes of w_i = (M / p_i)
mod q and with c_i = round(2^14 / p_i), the limb sums assembled into S = sum_i y_i w_i, the
rounding t = floor(T / 2^14 + 1/2) of sum_i y_i / p_i, (-t M) mod q added, and the reduction
of x < 4081 q by the single-precision quotient estimate floor(x / q - 1/2) and one conditional
subtraction.  The products C are drawn over the whole range the moduli are chosen for,
|C| <= M / 4, ends included, and every result must be C mod q (Python integers).  This pins the
error analysis the kernel rests on; the GPU tests check the kernel itself."""
import os
import re

import numpy as np
import pytest

_HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2503_16080_amd", "csrc", "crt.hpp")


def _moduli():
    text = open(_HDR).read()
    body = re.search(r"kCrtModuli\[kCrtMaxModuli\]\s*=\s*\{([^}]*)\}", text).group(1)
    return [int(v) for v in body.replace("\n", " ").split(",") if v.strip()]


MODULI = _moduli()
QS = [3, 5, 257, 65537, (1 << 50) - 27, (1 << 51) + 1 + (1 << 17) * 5, (1 << 52) - 47]
U32, U64 = (1 << 32) - 1, (1 << 64) - 1


def _dot4(a_bytes, b_bytes, acc):
    """v_dot4_u32_u8 without clamping: the sum of the four byte products plus acc, mod 2^32."""
    return (acc + sum(x * y for x, y in zip(a_bytes, b_bytes))) & U32


def recombine(y, D, q):
    """The kernel's steps for one entry: y holds the D coefficients y_i in [0, p_i)."""
    G = (D + 3) // 4
    p = MODULI[:D]
    M = 1
    for v in p:
        M *= v
    w = [(M // v) % q for v in p] + [0] * (4 * G - D)
    c = [(32768 + v) // (2 * v) for v in p] + [0] * (4 * G - D)  # round(2^14 / p_i)
    assert max(c) <= 255
    yy = list(y) + [0] * (4 * G - D)
    limbs = []
    for l in range(7):
        acc = 0
        for g in range(G):
            acc = _dot4(yy[4 * g:4 * g + 4], [(w[4 * g + j] >> (8 * l)) & 255 for j in range(4)], acc)
        assert acc < 1 << 20
        limbs.append(acc)
    T = 0
    for g in range(G):
        T = _dot4(yy[4 * g:4 * g + 4], c[4 * g:4 * g + 4], T)
    t = (T + 8192) >> 14
    assert 0 <= t <= D
    A = limbs[0] + (limbs[1] << 8)
    B = limbs[2] + (limbs[3] << 8)
    H = limbs[4] + (limbs[5] << 8) + (limbs[6] << 16)
    assert A <= U32 and B <= U32 and H <= U32
    X = A + (B << 16)
    S = X + (H << 32)
    assert S == sum(a * b for a, b in zip(yy, w)) and S + q <= U64
    negtm = (-t * (M % q)) % q
    x = S + negtm
    assert x < 4081 * q
    return reduce_small_quotient(x, q), t


def _f32(v):
    return float(np.float32(v))


def reduce_small_quotient(x, q):
    """x mod q for x < 4081 q: qt = floor(fl(fl(x) / q - 1/2)) in single precision, then
    r = x - qt q must lie in [0, 2 q).  1/q is taken one unit of 2^-24 either side of the
    correctly rounded reciprocal (the hardware reciprocal's error)."""
    x_lo, x_hi = x & U32, x >> 32
    xf = _f32(_f32(x_hi) * 4294967296.0 + _f32(x_lo))
    r0 = _f32(1.0 / _f32(q))
    out = None
    for qinv in (float(np.nextafter(np.float32(r0), np.float32(0))), r0,
                 float(np.nextafter(np.float32(r0), np.float32(1e30)))):
        tq = _f32(xf * qinv - 0.5)
        assert abs(tq - (x / q - 0.5)) < 0.01
        qt = int(max(tq, 0.0))
        r = x - qt * q
        assert 0 <= r < 2 * q, (x, q, qt)
        r = r - q if r >= q else r
        assert out is None or r == out
        out = r
    return out


@pytest.mark.parametrize("D", [8, 10, 11, 12, 14, 16])
def test_recombination_exact_over_the_whole_range(D):
    p = MODULI[:D]
    M = 1
    for v in p:
        M *= v
    s = [pow(M // v, -1, v) for v in p]
    rng = np.random.default_rng(4200 + D)
    quarter = M // 4
    Cs = [quarter, -quarter, quarter - 1, -quarter + 1, 0, 1, -1]
    Cs += [int(v) for v in rng.integers(-(1 << 62), 1 << 62, size=200)]
    # uniform over [-M/4, M/4] from four 32-bit draws per value (M exceeds 2^64)
    for _ in range(400):
        r = 0
        for _ in range(5):
            r = (r << 32) | int(rng.integers(0, 1 << 32))
        Cs.append(r % (2 * quarter + 1) - quarter)
    for q in QS:
        for C in Cs:
            y = [(C * si) % v for si, v in zip(s, p)]
            got, t = recombine(y, D, q)
            assert got == C % q, (D, q, C, got)
            # t is the integer nearest sum_i y_i / p_i (within 1/4 of it)
            assert sum(yi * (M // v) for yi, v in zip(y, p)) - t * M == C


def test_largest_coefficients_stay_in_range():
    """Every y_i = p_i - 1 (the largest sums, whatever product they come from): the limb sums,
    the 64-bit sum plus the table entry and the rounding stay within their registers."""
    for D in (8, 10, 11, 12, 14, 16):
        for q in QS:
            y = [v - 1 for v in MODULI[:D]]
            G = (D + 3) // 4
            w = [q - 1] * D + [0] * (4 * G - D)
            S = sum(a * b for a, b in zip(y, w))
            assert S + q <= U64 and S + q - 1 < 4081 * q
            assert reduce_small_quotient(S + q - 1, q) == (S + q - 1) % q
            for l in range(7):
                assert sum(a * ((b >> (8 * l)) & 255) for a, b in zip(y, w)) < 1 << 20
            assert sum(a * ((32768 + v) // (2 * v)) for a, v in zip(y, MODULI[:D])) + 8192 < 1 << 32
