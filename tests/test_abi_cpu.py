"""CPU-only checks of the C ABI: the library loads, exports every declared symbol, and its
host logic (argument checks, exactness planner) behaves as documented -- no device calls."""
import ctypes
import math
import os
import re

import pytest

import paper_2503_16080_amd as hlb
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hlb.h")

Q50 = wl.ntt_primes(50, 1)[0]  # the largest 50-bit prime = 1 (mod 2^17)


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hlb_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = hlb.load()
    names = _declared()
    assert "hlb_cp_mm" in names and "hlb_mod_pp_mm" in names and "hlb_cp_mm_batch" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    assert hlb.hlb_status_str(0) == "ok"
    assert "invalid" in hlb.hlb_status_str(1)
    assert hlb.hlb_status_str(99) == "unknown status"


def test_plan_int8_cpmm_matches_bounds():
    p = hlb.plan(1, 8192, Q50, 1 << 20, "int8")
    assert (p["form"], p["p_limbs"], p["x_limbs"], p["shifts"], p["limb_bits"]) == (2, 3, 7, 9, 8)
    # |c_s| <= pairs * k_chunk * 128^2 < 2^31, chunk a whole number of 64-byte K stages
    assert p["max_pairs"] == 3
    assert p["k_chunk"] % 64 == 0
    assert p["max_pairs"] * p["k_chunk"] * 128 * 128 < 2 ** 31
    assert p["max_pairs"] * (p["k_chunk"] + 64) * 128 * 128 >= 2 ** 31  # largest such chunk
    assert p["k_chunk"] >= 16384   # no fold for any benchmark shape
    assert p["acc_bound_log2"] < 31


def test_plan_int8_digit_counts():
    # 45-bit primes need 6 balanced digits (capacity 127 * (256^6 - 1) / 255 ~ 2^47)
    p = hlb.plan(1, 4096, (1 << 45) - 55, 1 << 20, "int8")
    assert (p["p_limbs"], p["x_limbs"]) == (3, 6)
    # a plaintext beyond 3 digits (capacity 8355711) or a full residue uses 7 x 7
    p = hlb.plan(1, 4096, Q50, 8355712, "int8")
    assert (p["p_limbs"], p["x_limbs"]) == (7, 7)
    p = hlb.plan(0, 256, Q50, 1, "int8")
    assert (p["p_limbs"], p["x_limbs"], p["shifts"], p["max_pairs"]) == (7, 7, 13, 7)
    assert 7 * p["k_chunk"] * 16384 < 2 ** 31
    cap = lambda D: 127 * (256 ** D - 1) // 255
    for q in [3, 97, 1 << 20, (1 << 45) + 1, Q50, (1 << 52) - 1]:
        p = hlb.plan(0, 64, q, 1, "int8")
        assert cap(p["x_limbs"]) >= q - 1


def test_plan_fp64_paper_form():
    # one plaintext limb (k2 = 1) and three ciphertext limbs (k1 = 3), as in Section 6.3
    p = hlb.plan(1, 8192, Q50, 1 << 20, "fp64")
    assert (p["form"], p["p_limbs"], p["x_limbs"]) == (1, 1, 3)
    w = p["limb_bits"]
    assert 3 * w >= 50
    assert p["k_chunk"] * (1 << 20) * ((1 << w) - 1) < 2 ** 53
    assert p["k_chunk"] >= 16384
    # general Mod-PP-MM: both operands in L limbs, L * k * (2^w - 1)^2 < 2^53
    p = hlb.plan(0, 256, Q50, 1, "fp64")
    L, w = p["p_limbs"], p["limb_bits"]
    assert L == p["x_limbs"] and L * w >= 50
    assert L * p["k_chunk"] * ((1 << w) - 1) ** 2 < 2 ** 53


def test_plan_auto_prefers_int8_and_forced_chunk():
    # AUTO takes the multimodular form when its moduli count is below 3/4 of the digit pairs
    # (11 < 15.75 for a 20-bit plaintext and 50-bit primes), the digit form when that fails
    # (k beyond the int32 bound of the multimodular products)
    assert hlb.plan(1, 4096, Q50, 1 << 20, "auto")["form"] == hlb.FORM_INT8_CRT
    assert hlb.plan(0, 4096, Q50, 1, "auto")["form"] == hlb.FORM_INT8_CRT
    assert hlb.plan(1, 200000, Q50, 1 << 20, "auto")["form"] == hlb.FORM_INT8
    assert hlb.plan(1, 4096, Q50, 1 << 51, "auto")["form"] == hlb.FORM_INT8_CRT   # 16 moduli vs 49 pairs
    try:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 200)
        assert hlb.plan(1, 4096, Q50, 1 << 20, "int8")["k_chunk"] == 192
        assert hlb.plan(1, 4096, Q50, 1 << 20, "fp64")["k_chunk"] == 192
    finally:
        hlb.set_option(hlb.OPT_FORCE_KCHUNK, 0)
    assert hlb.plan(1, 4096, Q50, 1 << 20, "int8")["k_chunk"] > 4096


def test_plan_rejects_bad_arguments():
    lib = hlb.load()
    d = hlb.PlanDesc()
    for args in [(2, 64, Q50, 1, 0), (0, -1, Q50, 1, 0), (0, 64, 1, 1, 0), (0, 64, 1 << 52, 1, 0),
                 (1, 64, Q50, 0, 0), (1, 64, Q50, 1 << 52, 0), (0, 64, Q50, 1, 7)]:
        assert lib.hlb_plan(*args, ctypes.byref(d)) == 1, args


def test_entry_points_reject_bad_arguments_before_device_work():
    lib = hlb.load()
    fake = 0x1000  # never dereferenced: every call below fails validation first
    # modulus out of range
    assert lib.hlb_mod_pp_mm(1, 4, 4, 4, fake, 4, fake, 4, fake, 4, 0, None) == 1
    assert lib.hlb_mod_pp_mm(1 << 52, 4, 4, 4, fake, 4, fake, 4, fake, 4, 0, None) == 1
    # negative sizes, short leading dimensions, null pointers
    assert lib.hlb_mod_pp_mm(97, -1, 4, 4, fake, 4, fake, 4, fake, 4, 0, None) == 1
    assert lib.hlb_mod_pp_mm(97, 4, 4, 4, fake, 3, fake, 4, fake, 4, 0, None) == 1
    assert lib.hlb_mod_pp_mm(97, 4, 4, 4, fake, 4, fake, 4, None, 4, 0, None) == 1
    assert lib.hlb_mod_pp_mm(97, 4, 4, 4, None, 4, fake, 4, fake, 4, 0, None) == 1
    # empty products are no-ops that touch nothing
    assert lib.hlb_mod_pp_mm(97, 0, 4, 4, None, 4, None, 4, None, 4, 0, None) == 0
    assert lib.hlb_mod_pp_mm(97, 4, 4, 0, None, 4, None, 4, None, 4, 0, None) == 0
    qs = (ctypes.c_uint64 * 2)(Q50, 1)
    assert lib.hlb_cp_mm(4, 4, 4, 4, fake, 4, 8, fake, fake, qs, 2, fake, fake, 2, None) == 1
    qs = (ctypes.c_uint64 * 1)(Q50)
    assert lib.hlb_cp_mm(4, 4, 4, 4, fake, 4, -1, fake, fake, qs, 1, fake, fake, 2, None) == 1
    assert lib.hlb_cp_mm(4, 4, 4, 4, fake, 4, 1 << 52, fake, fake, qs, 1, fake, fake, 2, None) == 1
    assert lib.hlb_cp_mm(4, 4, 4, 4, fake, 2, 8, fake, fake, qs, 1, fake, fake, 2, None) == 1
    assert lib.hlb_cp_mm(4, 4, 4, 4, fake, 4, 8, fake, fake, None, 1, fake, fake, 2, None) == 1
    assert lib.hlb_cp_mm(4, 4, 4, 4, fake, 4, 8, fake, fake, qs, 0, fake, fake, 2, None) == 0
    assert lib.hlb_cp_mm(0, 4, 4, 4, fake, 4, 8, fake, fake, qs, 1, fake, fake, 2, None) == 0
    assert lib.hlb_cp_mm(4, 4, 4, 4, fake, 4, 8, fake, fake, qs, 1, None, fake, 2, None) == 1
    assert lib.hlb_cp_mm_batch(None, 3, qs, 1, 2, None) == 1
    assert lib.hlb_cp_mm_batch(None, 0, qs, 1, 2, None) == 0
    assert lib.hlb_cp_mm_trunc_b(4, 4, 4, 4, fake, 4, -1, fake, fake, qs, 1, fake, fake, 40.0, 2, None) == 1
    qs2 = (ctypes.c_uint64 * 2)(Q50, Q50 - 2)
    assert lib.hlb_cp_mm_trunc_b(4, 4, 4, 4, fake, 4, 8, fake, fake, qs2, 2, fake, fake, 40.0, 2, None) == 1
    assert lib.hlb_cp_mm_trunc_b(4, 4, 4, 4, fake, 2, 8, fake, fake, qs, 1, fake, fake, 40.0, 2, None) == 1
    assert lib.hlb_cp_mm_trunc_b(4, 4, 4, 4, fake, 4, 8, fake, fake, qs, 0, fake, fake, 40.0, 2, None) == 0
    assert lib.hlb_cp_mm_trunc_b(4, 4, 4, 4, fake, 4, 8, fake, fake, qs, 1, fake, None, 40.0, 2, None) == 1
    bad = ctypes.c_int64(0)
    assert lib.hlb_validate_residues(fake, 4, 4, 3, 97, ctypes.byref(bad), None) == 1
    assert lib.hlb_validate_residues(fake, 0, 4, 4, 97, ctypes.byref(bad), None) == 0
    assert bad.value == -1
    assert lib.hlb_set_option(999, 1) == 6
    assert lib.hlb_set_option(hlb.OPT_FORCE_KCHUNK, -5) == 1
    assert lib.hlb_set_option(hlb.OPT_F64_PLANES, 0) == 0 and lib.hlb_set_option(hlb.OPT_F64_PLANES, 1) == 0
    for v in (0, 1, 2, -1):
        assert lib.hlb_set_option(hlb.OPT_CRT_WIDE, v) == 0
    assert lib.hlb_set_option(hlb.OPT_CRT_WIDE, 3) == 1 and lib.hlb_set_option(hlb.OPT_CRT_WIDE, -2) == 1
    assert lib.hlb_set_option(hlb.OPT_WS_CAP, -1) == 1
    assert lib.hlb_set_option(hlb.OPT_WS_CAP, 1 << 20) == 0 and lib.hlb_set_option(hlb.OPT_WS_CAP, 0) == 0


def test_no_silent_fallback_without_library(monkeypatch):
    monkeypatch.setattr(hlb, "_lib", None)
    monkeypatch.setattr(hlb, "_LIB_PATH", "/nonexistent/libhlb.so")
    with pytest.raises(hlb.HlbError):
        hlb.load()


def test_tile_class_heuristic_and_tuning_table(tmp_path):
    # padding-waste heuristic: 64-row problems take the 64 x 128 class, square ones 128 x 64
    assert hlb.hlb_tune_class(7, 64, 1024, 1024) == 1
    assert hlb.hlb_tune_class(7, 8192, 8192, 8192) == 0
    assert hlb.hlb_tune_class(6, 60, 4096, 512) == 1    # pads to 64 rows instead of 128
    assert hlb.hlb_tune_class(6, 100, 4096, 512) == 0   # both classes pad to 128 rows
    # table entries override the heuristic for their bucket only
    hlb.hlb_tune_set(7, 13, 13, 13, 1)
    try:
        assert hlb.hlb_tune_class(7, 8192, 8192, 8192) == 1
        assert hlb.hlb_tune_class(7, 8192, 8192, 4096) == 0
    finally:
        hlb.hlb_tune_set(7, 13, 13, 13, -1)
    assert hlb.hlb_tune_class(7, 8192, 8192, 8192) == 0
    f = tmp_path / "tune.txt"
    f.write_text("# comment\n6 6 10 10 0\nnot a line\n")
    hlb.hlb_tune_load(str(f))
    try:
        assert hlb.hlb_tune_class(6, 64, 1024, 1024) == 0
    finally:
        hlb.hlb_tune_set(6, 6, 10, 10, -1)
    assert hlb.hlb_tune_class(6, 64, 1024, 1024) == 1
    with pytest.raises(hlb.HlbError):
        hlb.hlb_tune_set(7, 1, 1, 1, 5)
    with pytest.raises(hlb.HlbError):
        hlb.hlb_tune_load(str(tmp_path / "missing.txt"))
    try:
        hlb.set_option(hlb.OPT_FORCE_CLASS, 0)
        assert hlb.hlb_tune_class(7, 64, 1024, 1024) == 0
    finally:
        hlb.set_option(hlb.OPT_FORCE_CLASS, -1)
    with pytest.raises(hlb.HlbError):
        hlb.set_option(hlb.OPT_FORCE_CLASS, 2)


def test_multimodular_tile_class_table(tmp_path):
    # no entry: the widest class (256 x 384); entries per (moduli, log2 m, log2 n, log2 k)
    assert hlb.hlb_tune_class_crt(10, 300, 1000, 1000) == 2
    hlb.hlb_tune_set_crt(10, 8, 9, 9, 0)
    try:
        assert hlb.hlb_tune_class_crt(10, 300, 1000, 1000) == 0
        assert hlb.hlb_tune_class_crt(11, 300, 1000, 1000) == 2   # another moduli count
        assert hlb.hlb_tune_class_crt(10, 600, 1000, 1000) == 2   # another row bucket
        # the digit form's entries live beside them without clashing
        assert hlb.hlb_tune_class(7, 300, 1000, 1000) in (0, 1)
        # a forced class overrides the table, -1 returns to it
        hlb.set_option(hlb.OPT_CRT_WIDE, 1)
        assert hlb.hlb_tune_class_crt(10, 300, 1000, 1000) == 1
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
        assert hlb.hlb_tune_class_crt(10, 300, 1000, 1000) == 0
    finally:
        hlb.set_option(hlb.OPT_CRT_WIDE, -1)
        hlb.hlb_tune_set_crt(10, 8, 9, 9, -1)
    assert hlb.hlb_tune_class_crt(10, 300, 1000, 1000) == 2
    # the table file holds both kinds of lines
    f = tmp_path / "tune.txt"
    f.write_text("# comment\ncrt 10 6 7 7 1   # ms\n6 6 10 10 0\ncrt 99 6 7 7 1\ncrt 10 6 7 7 5\n")
    hlb.hlb_tune_load(str(f))
    try:
        assert hlb.hlb_tune_class_crt(10, 100, 200, 200) == 1
        assert hlb.hlb_tune_class(6, 64, 1024, 1024) == 0
    finally:
        hlb.hlb_tune_set_crt(10, 6, 7, 7, -1)
        hlb.hlb_tune_set(6, 6, 10, 10, -1)
    assert hlb.hlb_tune_class_crt(10, 100, 200, 200) == 2
    for bad in ((0, 1, 1, 1, 0), (17, 1, 1, 1, 0), (10, 64, 1, 1, 0), (10, 1, 1, 1, 3), (10, 1, 1, 1, -2)):
        with pytest.raises(hlb.HlbError):
            hlb.hlb_tune_set_crt(*bad)
    assert hlb.hlb_tune_class_crt(0, 1, 1, 1) == -1 and hlb.hlb_tune_class_crt(10, 0, 1, 1) == -1


def test_trunc_b_planner_bounds():
    # INT8: the largest number of dropped shifts (<= 3) whose bound
    # k 2^14 sum_{s<drop} pairs(s) 256^s fits the budget and stays below q_min / 2
    import math
    pairs = lambda s, dp, dx: sum(1 for i in range(dp) if 0 <= s - i < dx)
    for k, bits, dx in ((8192, 50, 7), (4096, 45, 6), (300, 50, 7)):
        q = wl.ntt_primes(bits, 1)[0]
        for budget in (20.0, 27.5, 36.5, 40.0, 45.0, 60.0):
            want = 0
            for drop in (3, 2, 1):
                b = k * 2 ** 14 * sum(pairs(s, 3, dx) * 256 ** s for s in range(drop))
                if math.log2(b) <= budget and b < q / 2:
                    want = drop
                    break
            p = hlb.plan_trunc_b(k, q, q, 1 << 20, budget, "int8")
            assert p["dropped_shifts"] == want and p["truncated"] == (want > 0)
            assert p["products"] == 3 * dx - sum(pairs(s, 3, dx) for s in range(want))
    # no truncation when the K range needs a fold
    assert hlb.plan_trunc_b(50000, Q50, Q50, 1 << 20, 60.0, "int8")["truncated"] == 0
    # FP64: (k + 2) 2^-52 k pmax (q/2)
    k, q, pm = 8192, Q50, 1 << 20
    p = hlb.plan_trunc_b(k, q, q, pm, 45.0, "fp64")
    assert p["truncated"] and p["products"] == 1
    assert abs(p["err_bound_log2"] - math.log2((k + 2) * 2.0 ** -52 * k * pm * (q // 2))) < 1e-9
    assert not hlb.plan_trunc_b(k, q, q, pm, 42.0, "fp64")["truncated"]
    assert not hlb.plan_trunc_b(1 << 20, q, q, 1 << 32, 200.0, "fp64")["truncated"]  # k pmax > 2^51
    with pytest.raises(hlb.HlbError):
        hlb.plan_trunc_b(10, Q50, 7, 1, 40.0, "int8")   # q_min > q_max


def test_crt_plan_moduli_count():
    # the smallest number of the fixed coprime moduli whose product is at least 4 |V|,
    # |V| <= k * a * floor(q/2), rounded up to an instantiated count
    import math
    mods = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191]
    for a_ in range(len(mods)):
        for b_ in range(a_ + 1, len(mods)):
            assert math.gcd(mods[a_], mods[b_]) == 1
    inst = [8, 10, 11, 12, 14, 16]
    for kind, k, q, pm in ((1, 8192, Q50, 1 << 20), (1, 256, Q50, 1 << 20), (0, 8192, Q50, 1),
                           (1, 4096, wl.ntt_primes(45, 1)[0], 1 << 20), (0, 100, 97, 1)):
        a = pm if kind == 1 else q // 2
        need = math.log2(k) + math.log2(a) + math.log2(max(q // 2, 1)) + 2
        D, have = 0, 0.0
        while have < need:
            have += math.log2(mods[D])
            D += 1
        D = min(d for d in inst if d >= D)
        p = hlb.plan(kind, k, q, pm, "int8_crt")
        assert p["form"] == 3 and p["p_limbs"] == D
    with pytest.raises(hlb.HlbError):
        hlb.plan(1, 131072, Q50, 1 << 20, "int8_crt")


def test_binding_rejects_mismatched_tensors_before_device_work():
    # Shapes are checked before devices, so CPU (and meta) tensors of the wrong shape raise
    # ValueError without any device call; correctly shaped CPU tensors then raise TypeError
    # (they are not device memory) instead of reaching the library.
    import torch

    def z(*shape, dtype=torch.int64):
        return torch.zeros(shape, dtype=dtype, device="meta")

    q = [Q50, Q50 - 2]
    L, m, k, n = 2, 8, 6, 5
    P, A, B = z(m, k), z(L, k, n), z(L, k, n)
    # undersized, transposed or wrongly batched outputs of cp_mm / cp_mm_trunc_b
    for PA, PB in [(z(L, m, n - 1), z(L, m, n)), (z(L, m, n), z(L, m - 1, n)), (z(1, m, n), z(L, m, n)),
                   (z(L, n, m), z(L, m, n)), (z(L * m * n), z(L, m, n))]:
        with pytest.raises(ValueError):
            hlb.cp_mm(P, A, B, q, p_absmax=1, out=(PA, PB))
    for PA, PB in [(z(1, m, n - 1), z(1, m, n)), (z(1, m, n), z(1, m + 1, n)), (z(2, m, n), z(1, m, n))]:
        with pytest.raises(ValueError):
            hlb.cp_mm_trunc_b(P, A[:1], B[:1], [Q50], 40.0, p_absmax=1, out=(PA, PB))
    # short or mis-sized ciphertext parts
    with pytest.raises(ValueError):
        hlb.cp_mm(P, z(L, k - 1, n), B, q)
    with pytest.raises(ValueError):
        hlb.cp_mm(P, A, z(L + 1, k, n), q)
    with pytest.raises(ValueError):
        hlb.cp_mm(z(m * k), A, B, q)
    # wrong dtype is a TypeError
    with pytest.raises(TypeError):
        hlb.cp_mm(P, A, B, q, out=(z(L, m, n, dtype=torch.int32), z(L, m, n)))
    # mod_pp_mm: out must be m x n
    with pytest.raises(ValueError):
        hlb.mod_pp_mm(Q50, z(m, k), z(k, n), out=z(m, n + 1))
    with pytest.raises(ValueError):
        hlb.mod_pp_mm(Q50, z(m, k), z(k + 1, n))
    # batch: every member's A, B, PA, PB against its P and the prime count
    good = dict(P=P, A=A, B=B)
    for bad in [dict(P=P, A=z(L, k + 1, n), B=B), dict(P=P, A=A, B=z(L, k, n)[0]),
                dict(P=P, A=z(L + 1, k, n), B=B), dict(P=P, A=A, B=B, PA=z(L, m - 1, n)),
                dict(P=P, A=A, B=B, PB=z(L, m, n + 3)), dict(P=z(m, k, 1), A=A, B=B)]:
        with pytest.raises(ValueError):
            hlb.cp_mm_batch([good, bad], q)
    # ccmm core and the test helpers
    with pytest.raises(ValueError):
        hlb.ccmm_pp_core(z(L, m, k), z(L, m, k), z(L, k, n), z(L, k + 1, n), q)
    with pytest.raises(ValueError):
        hlb.hlb_test_encrypt(z(L, k, n), z(n, n - 1), z(k, n), q)
    with pytest.raises(ValueError):
        hlb.hlb_test_encrypt(z(L, k, n), z(n, n), z(k - 1, n), q)
    with pytest.raises(ValueError):
        hlb.hlb_test_decrypt(z(L, m, n), z(L, m - 1, n), z(n, n), q)
    # correct shapes on the CPU: refused as non-device tensors, never passed to the library
    c = lambda *s: torch.zeros(s, dtype=torch.int64)
    with pytest.raises(TypeError):
        hlb.cp_mm(c(m, k), c(L, k, n), c(L, k, n), q, out=(c(L, m, n), c(L, m, n)))
    with pytest.raises(TypeError):
        hlb.cp_mm_batch([dict(P=c(m, k), A=c(L, k, n), B=c(L, k, n))], q)


def test_environment_form_switch_and_validate_option():
    """HLB_FORM sets the form of calls that pass HLB_FORM_AUTO (hlb_plan included) and leaves
    explicit forms alone; HLB_OPT_VALIDATE is a host-side option (accepted without a GPU).  The
    environment is read once per process, so each setting runs in a fresh interpreter."""
    import json
    import subprocess
    import sys
    q = wl.ntt_primes(50, 1)[0]
    code = ("import json, paper_2503_16080_amd as h; "
            f"print(json.dumps([h.plan(1, 8192, {q}, 1 << 20, 'auto')['form'], "
            f"h.plan(1, 8192, {q}, 1 << 20, 'int8')['form']]))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    got = {}
    for env_form in (None, "fp64", "int8", "int8_crt", "auto", "bogus"):
        env = dict(os.environ)
        env.pop("HLB_FORM", None)
        if env_form is not None:
            env["HLB_FORM"] = env_form
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr
        got[env_form] = json.loads(r.stdout.strip().splitlines()[-1])
    # auto picks the multimodular form at d = 8192; an unknown name is ignored
    assert got[None] == [hlb.FORM_INT8_CRT, hlb.FORM_INT8]
    assert got["fp64"] == [hlb.FORM_FP64, hlb.FORM_INT8]
    assert got["int8"] == [hlb.FORM_INT8, hlb.FORM_INT8]
    assert got["int8_crt"] == [hlb.FORM_INT8_CRT, hlb.FORM_INT8]
    assert got["auto"] == got[None] and got["bogus"] == got[None]
    hlb.set_option(hlb.OPT_VALIDATE, 1)
    hlb.set_option(hlb.OPT_VALIDATE, 0)
