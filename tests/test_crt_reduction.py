"""The reductions c mod p of the multimodular GEMM's epilogue, emulated on the CPU in the
arithmetic the kernel performs (single-precision products rounded to nearest, 24-bit integer
multiply-adds, unsigned minima), over every modulus from 191 to 256 and the products that reach
the edge of each one's range: the short form for |c| <= 2^28, the general one for every int32 c.
These pin the error analysis the kernel rests on; the GPU tests check the kernel itself."""
import numpy as np

MODULI = range(191, 257)


def _windows(lo, hi, width, rng, extra):
    """c near both ends of [lo, hi] and around zero, plus `extra` uniform samples."""
    return np.concatenate([np.arange(lo, lo + width), np.arange(hi - width + 1, hi + 1),
                           np.arange(-width, width), rng.integers(lo, hi + 1, size=extra)]).astype(np.int64)


def _check(c, p, y):
    want = np.mod(c, p)
    bad = np.flatnonzero(y != want)
    assert bad.size == 0, (p, c[bad[:4]], y[bad[:4]], want[bad[:4]])


def short_form(c, p):
    # x = fl(fl(c) fl(1/p)); t = floor(x + 1/2); r = c - t p in [-p, p); canonical by one minimum
    pinv = np.float32(1) / np.float32(p)
    x = c.astype(np.float32) * pinv
    # the conversion's x + 1/2, exact or rounded to single precision: either is within range
    for t in (np.floor(x.astype(np.float64) + 0.5), np.floor(x + np.float32(0.5))):
        t = t.astype(np.int64)
        assert np.abs(t).max() < (1 << 23)  # the 24-bit multiply-add's operand range
        r = c - t * p
        assert r.min() >= -p and r.max() < p
    return np.where(r < 0, r + p, r)


def general_form(c, p):
    # u = h (2^16 mod p) + l = c (mod p); t = floor(fl(fl(u) fl(1/p))); r = u - t p in [-p, 2p)
    h, l = c >> 16, c & 0xFFFF
    u = h * ((1 << 16) % p) + l
    assert np.abs(u).max() < (1 << 23) + (1 << 16)
    pinv = np.float32(1) / np.float32(p)
    t = np.floor(u.astype(np.float32) * pinv).astype(np.int64)
    r = u - t * p
    assert r.min() >= -p and r.max() < 2 * p
    r = np.where(r < 0, r + p, r)
    return np.where(r >= p, r - p, r)


def test_short_form_exact_up_to_2_28():
    rng = np.random.default_rng(1)
    c = _windows(-(1 << 28), 1 << 28, 1 << 16, rng, 1 << 17)
    for p in MODULI:
        _check(c, p, short_form(c, p))


def test_general_form_exact_for_every_int32():
    rng = np.random.default_rng(2)
    c = _windows(-(1 << 31), (1 << 31) - 1, 1 << 16, rng, 1 << 17)
    for p in MODULI:
        _check(c, p, general_form(c, p))
